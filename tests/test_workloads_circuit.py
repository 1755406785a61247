"""Pins of the circuit bond-matrix generator (the paper's introductory
circuit, Sec. 1 footnote 1) and of the closed form its tests use.

* trace 1 exactly; the integer matrix R behind rho = R / 2^n has rank <= 2
  (checked exactly: every 3x3 minor of a sample is zero in integers);
* across the last cut the eigenvalues are exactly 1 - 2^(-n+1) and 2^(-n+1)
  (characteristic polynomial of the 2x2 matrix in rationals);
* a rank-2 density matrix has nonzero eigenvalues (1 +- sqrt(2F - 1)) / 2 with
  F = ||rho||_F^2: checked against the MPFR oracle to 1e-60 on every cut of a
  6-qubit state (orders up to 8), which also pins the oracle on this family.
"""
import itertools
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W


def closed_form_pair(R, n):
    """The two nonzero eigenvalues of rho = R / 2^n (rank 2, trace 1), as Decimals."""
    getcontext().prec = 90
    F = Fraction(int((R.astype(object) ** 2).sum()), 4 ** n)
    disc = Decimal((2 * F - 1).numerator) / Decimal((2 * F - 1).denominator)
    r = disc.sqrt()
    return (1 - r) / 2, (1 + r) / 2


@pytest.mark.parametrize("n", [4, 9, 14])
def test_trace_rank_and_last_cut(n):
    for m in W.circuit_bond_matrices(n, seed=3):
        R = m["R"].astype(object)
        assert sum(R[i, i] for i in range(R.shape[0])) == 2 ** n
        d = R.shape[0]
        if d >= 3:
            rng = np.random.default_rng(d)
            for _ in range(20):
                rows = sorted(rng.choice(d, 3, replace=False))
                cols = sorted(rng.choice(d, 3, replace=False))
                M = [[R[i, j] for j in cols] for i in rows]
                det = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
                       - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                       + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]))
                assert det == 0
    last = W.circuit_bond_matrices(n, seed=3)[-1]
    R = last["R"].astype(object)
    assert R.shape == (2, 2)
    tr = Fraction(R[0, 0] + R[1, 1], 2 ** n)
    det = Fraction(R[0, 0] * R[1, 1] - R[0, 1] * R[1, 0], 4 ** n)
    eps = Fraction(1, 2 ** (n - 1))
    # eps and 1 - eps are the roots of x^2 - tr x + det
    assert tr == 1 and det == eps * (1 - eps)


def test_closed_form_against_oracle():
    n = 6
    for m in W.circuit_bond_matrices(n, seed=5):
        rho = m["rho"]
        ref = oracle.heev([rho], want_vectors=False).w_limbs
        lo, hi = closed_form_pair(m["R"], n)
        got = [sum((Fraction(float(x)) for x in ref[:, k]), Fraction(0)) for k in range(rho.shape[0])]
        got.sort()
        assert abs(Decimal(got[-1].numerator) / Decimal(got[-1].denominator) - hi) < Decimal("1e-60")
        assert abs(Decimal(got[-2].numerator) / Decimal(got[-2].denominator) - lo) < Decimal("1e-60")
        for x in got[:-2]:
            assert abs(x) < Fraction(1, 10 ** 60)
