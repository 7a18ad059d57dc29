"""Planted mistakes in the oracle must fail its pins (CPU only).

Each case copies ks_oracle.c, plants one plausible mistake (a dropped term, a
wrong sign, a transposed operand, an off-by-one step index) in the QR sweep,
the back-substitution, or either covariance recursion (square-root RTS over
R; information-form RTS over the model matrices), compiles the copy with gcc into a temporary directory and checks that the
dense-definition pin used in test_oracle_pins.py (states, both covariance
forms, lag-one blocks) no longer holds for at least one small probe problem.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import build as obuild
from oracle import dense, seq
from paper_2502_11686_amd import gen

MUTANTS = {
    "B sign flipped": ("row[s] = -Fi[r * n + s];", "row[s] = Fi[r * n + s];"),
    "smoother term dropped (square-root form)": ("Sjj[r * n + s] = Ri[r * n + s] - acc;", "Sjj[r * n + s] = Ri[r * n + s];"),
    "gain transposed in S_{i,i+1}": ("acc += T[r * n + q] * Snext[q * n + s];",
                             "acc += T[q * n + r] * Snext[q * n + s];"),
    "c dropped": ("row[2 * n] = c[(size_t)i * n + r];", "row[2 * n] = 0.0 * c[(size_t)i * n + r];"),
    "R_i,i+1 transposed in back-sub": ("y[r] -= Rsi[r * n + s] * yn[s];", "y[r] -= Rsi[s * n + r] * yn[s];"),
    "Householder tau sign": ("double tau = (beta - alpha) / beta;", "double tau = (alpha - beta) / beta;"),
    "diag whitening power": ("double s = 1.0 / sqrt(cov[r]);", "double s = 1.0 / cov[r];"),
    "H transposed": ("H[(size_t)i * nn + r * n + s]", "H[(size_t)i * nn + s * n + r]"),
    "forward-substitution sign": ("X[r * ldx + c] -= l * X[s * ldx + c];", "X[r * ldx + c] += l * X[s * ldx + c];"),
    "G step off by one": ("G + ((size_t)i * m + r) * n", "G + ((size_t)(i ? i - 1 : 0) * m + r) * n"),
    "F step off by one": ("const double *Fi = F + (size_t)i * nn;",
                          "const double *Fi = F + (size_t)(i + 1 < k ? i + 1 : i) * nn;"),
    "R^-T R^-1 for R^-1 R^-T": ("acc += T[r * n + q] * T[s * n + q];", "acc += T[q * n + r] * T[q * n + s];"),
    "carried rows dropped": ("memcpy(S1, P, sizeof(double) * (size_t)p * w1);",
                             "memset(S1, 0, sizeof(double) * (size_t)p * w1);"),
    # the RTS covariance recursion
    "RTS Schur term sign": ("Lam[a * n + b] -= acc;", "Lam[a * n + b] += acc;"),
    "RTS smoother term dropped": ("Snew[a * n + b] = Li[a * n + b] + acc;", "Snew[a * n + b] = Li[a * n + b];"),
    "RTS gain with N transposed": ("acc += Li[a * n + q] * Nnext[q * n + b];",
                                   "acc += Li[a * n + q] * Nnext[b * n + q];"),
    "RTS H^T K^-1 H without H": ("xt_a_y(Hi, n, n, Cov, Hi, n, tmp);", "xt_a_y(Hi, n, n, Cov, Ident, n, tmp);"),
    "RTS F^T K^-1 F dropped": ("xt_a_y(Fn, n, n, Cov, Fn, n, tmp);",
                               "xt_a_y(Fn, n, n, Cov, Fn, n, tmp); memset(tmp, 0, sizeof(double) * nn);"),
    "RTS F of the previous step": ("const double *Fn = F + (size_t)i * nn;",
                                   "const double *Fn = F + (size_t)(i ? i - 1 : 0) * nn;"),
    "RTS observation of the previous step": (
        "xt_a_y(G + (size_t)i * m * n, m, n, Cov, G + (size_t)i * m * n, n, tmp);",
        "xt_a_y(G + (size_t)(i ? i - 1 : 0) * m * n, m, n, Cov, G + (size_t)(i ? i - 1 : 0) * m * n, n, tmp);"),
    "RTS lag-one block transposed": ("acc += Mi[a * n + q] * Sig[q * n + b];",
                                     "acc += Mi[q * n + a] * Sig[q * n + b];"),
}


def probes():
    out = []
    for seed, (k, n, m, cov, H) in enumerate([(7, 3, 2, "dense", "random"), (6, 2, 3, "diag", "identity"),
                                               (9, 4, 2, "dense", "identity")]):
        out.append(gen.make_problem(np.random.default_rng(500 + seed), k, n, m, cov=cov, H_mode=H))
    return out


def pins_hold(lib):
    """Both covariance forms (square-root RTS over R; information-form RTS), the
    states and the lag-one blocks against the dense definition."""
    for p in probes():
        d = dense.smooth(p)
        for from_rts in (False, True):
            o = seq.smooth(p, lib=lib, check=False, want_lag1=True, rts=from_rts)
            if o["status"] != seq.OK:
                return False
            eu = np.max(np.abs(o["u"] - d["u"])) / np.max(np.abs(d["u"]))
            es = np.max(np.linalg.norm(o["cov"] - d["cov"], axis=(1, 2)) / np.linalg.norm(d["cov"], axis=(1, 2)))
            el = max(np.linalg.norm(o["lag1"][i] - d["S"][i * p.n:(i + 1) * p.n, (i + 1) * p.n:(i + 2) * p.n])
                     / np.linalg.norm(d["cov"][i]) for i in range(p.k))
            if not (eu < 1e-11 and es < 1e-10 and el < 1e-10):
                return False
    return True


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_unmutated_copy_passes(tmp_path):
    lib = seq.load(obuild.build(src=obuild.SRC, out=str(tmp_path / "orig.so")))
    assert pins_hold(lib)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(obuild.SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/absent: {old}"
    mutated = tmp_path / "ks_oracle.c"
    mutated.write_text(src.replace(old, new))
    shutil.copy(os.path.join(obuild.HERE, "ks_oracle.h"), tmp_path / "ks_oracle.h")
    so = str(tmp_path / "mut.so")
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-I", str(tmp_path),
                    str(mutated), "-o", so, "-lm"], check=True)
    assert not pins_hold(seq.load(so)), f"pins did not catch: {name}"
