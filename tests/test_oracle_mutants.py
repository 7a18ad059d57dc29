"""Planted mistakes in the oracle must fail its pins (CPU only).

Each case copies ks_oracle.c, plants one plausible mistake (a dropped term, a
wrong sign, a transposed operand, an off-by-one step index), compiles the copy
with gcc into a temporary directory and checks that the dense-definition pin used
in test_oracle_pins.py no longer holds for at least one small probe problem.
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
    "SelInv term dropped": ("Sjj[r * n + s] = Ri[r * n + s] - acc;", "Sjj[r * n + s] = Ri[r * n + s];"),
    "T transposed in S_jI": ("acc += T[r * n + q] * Snext[q * n + s];",
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
}


def probes():
    out = []
    for seed, (k, n, m, cov, H) in enumerate([(7, 3, 2, "dense", "random"), (6, 2, 3, "diag", "identity"),
                                               (9, 4, 2, "dense", "identity")]):
        out.append(gen.make_problem(np.random.default_rng(500 + seed), k, n, m, cov=cov, H_mode=H))
    return out


def pins_hold(lib):
    for p in probes():
        d = dense.smooth(p)
        o = seq.smooth(p, lib=lib, check=False)
        if o["status"] != seq.OK:
            return False
        eu = np.max(np.abs(o["u"] - d["u"])) / np.max(np.abs(d["u"]))
        es = np.max(np.linalg.norm(o["cov"] - d["cov"], axis=(1, 2)) / np.linalg.norm(d["cov"], axis=(1, 2)))
        if not (eu < 1e-11 and es < 1e-10):
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
