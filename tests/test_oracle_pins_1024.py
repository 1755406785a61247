"""Pins of the MPFR oracle at 1024 bits with 16-limb results (the checker of
the precision beyond quad-double), against facts that do not depend on the
oracle itself:

* the paper's Schmidt pair (Sec. 1, footnote 1) far below quad-double:
  eigenvalues exactly 1 - eps and eps with eps = 2^-k up to k = 900,
  eigenvectors (1, +-conj(w))/sqrt 2;
* exact-spectrum Hadamard matrices whose dyadic spectra span 700 bits (inputs
  of up to 16 limbs): eigenvalues exact, eigenspaces exact;
* n <= 4: roots of the exact rational characteristic polynomial (mpmath at
  330 digits);
* trace(H) = sum(lam) and ||H||_F^2 = sum(lam^2) in exact rationals;
* agreement with the 256-bit oracle at the latter's resolution;
* the planted mistakes of the 256-bit pins, caught at 1024 bits too.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
import workloads as W

from test_oracle_pins import _charpoly_exact, _dyadic_spectrum

PREC = 1024
LIMBS = 16
TIGHT = Fraction(1, 2 ** 840)   # 16-limb (~2^-848 relative) output resolution


def _fr(limbs):
    return sum((Fraction(float(x)) for x in limbs), Fraction(0))


def _eigs(r):
    return [_fr(r.w_limbs[:, k]) for k in range(r.w_limbs.shape[1])]


def _vec(r, k):
    n = r.v_limbs.shape[1]
    out = []
    for i in range(n):
        re = sum(mpmath.mpf(float(r.v_limbs[l, i, k].real)) for l in range(r.v_limbs.shape[0]))
        im = sum(mpmath.mpf(float(r.v_limbs[l, i, k].imag)) for l in range(r.v_limbs.shape[0]))
        out.append(mpmath.mpc(re, im))
    return out


@pytest.mark.parametrize("k", [120, 300, 600, 900])
@pytest.mark.parametrize("omega", [1, -1j])
def test_schmidt_pair_exact_1024(k, omega):
    planes, (eps, one_minus) = W.schmidt_pair(k, omega, 2)
    r = oracle.heev(planes, prec=PREC, limbs=LIMBS)
    lam = _eigs(r)
    assert abs(lam[0] - eps) <= TIGHT
    assert abs(lam[1] - one_minus) <= TIGHT
    mpmath.mp.dps = 320
    w = mpmath.mpc(complex(omega).real, complex(omega).imag)
    for idx, sgn in ((1, 1), (0, -1)):
        v = _vec(r, idx)
        ex = [1 / mpmath.sqrt(2), sgn * mpmath.conj(w) / mpmath.sqrt(2)]
        ov = abs(mpmath.conj(ex[0]) * v[0] + mpmath.conj(ex[1]) * v[1])
        assert abs(ov - 1) < mpmath.mpf(2) ** -800


@pytest.mark.parametrize("n,limbs,span", [(16, 16, 700), (32, 8, 300)])
def test_hadamard_exact_1024(n, limbs, span):
    rng = np.random.Generator(np.random.PCG64(5000 + n + limbs))
    lam = _dyadic_spectrum(n, rng, span, mant_bits=40, zeros=2, dups=3)
    h = W.hadamard_exact(lam, seed=91 + n, limbs=limbs)
    r = oracle.heev(h.planes, prec=PREC, limbs=LIMBS)
    got = _eigs(r)
    scale = max(abs(x) for x in lam)
    for a, b in zip(got, h.lam):
        assert abs(a - b) <= scale * TIGHT
    # every vector of eigenvalue mu lies in the exact eigenspace of mu (binary64
    # evaluation of an exact-zero projection)
    Vx = h.vectors_unnormalised() / np.sqrt(n)
    V = r.v_limbs[0] + r.v_limbs[1]
    for mu in sorted(set(h.lam)):
        idx = [i for i, x in enumerate(h.lam) if x == mu]
        Q = Vx[:, idx]
        P = V[:, idx]
        assert np.abs(P - Q @ (Q.conj().T @ P)).max() < 1e-13


@pytest.mark.parametrize("n", [2, 3, 4])
def test_small_n_charpoly_roots_1024(n):
    A = W.random_elements(n, 40 + n)
    r = oracle.heev([A], prec=PREC, limbs=LIMBS)
    coeffs = _charpoly_exact(A)
    mpmath.mp.dps = 330
    roots = sorted(mpmath.re(z) for z in mpmath.polyroots([mpmath.mpf(x.numerator) / x.denominator for x in coeffs],
                                                          maxsteps=2000, extraprec=2000))
    for a, b in zip(_eigs(r), roots):
        assert abs(mpmath.mpf(a.numerator) / a.denominator - b) < mpmath.mpf(2) ** -820 * max(abs(x) for x in roots)


def test_invariants_1024():
    n = 24
    A = W.householder_hermitian(W.spectrum_c4(n), seed=W.seed_for(4, n) + 5)
    r = oracle.heev([A], prec=PREC, limbs=LIMBS, want_vectors=False)
    got = _eigs(r)
    tr = sum(Fraction(float(A[i, i].real)) for i in range(n))
    fro = Fraction(0)
    for i in range(n):
        for j in range(n):
            z = A[i, j] if i >= j else np.conj(A[j, i])
            re = Fraction(float(z.real))
            im = Fraction(0) if i == j else Fraction(float(z.imag))
            fro += re * re + im * im
    assert abs(sum(got) - tr) < Fraction(1, 2 ** 830)
    assert abs(sum(x * x for x in got) - fro) < Fraction(1, 2 ** 830)


def test_agrees_with_256_bit_oracle():
    A = W.random_elements(20, 77)
    hi = _eigs(oracle.heev([A], prec=PREC, limbs=LIMBS, want_vectors=False))
    lo = _eigs(oracle.heev([A], want_vectors=False))
    scale = max(abs(x) for x in hi)
    for a, b in zip(hi, lo):
        assert abs(a - b) <= scale * Fraction(1, 2 ** 205)


def _battery_1024():
    try:
        test_schmidt_pair_exact_1024(300, -1j)
        test_hadamard_exact_1024(32, 8, 300)
        test_small_n_charpoly_roots_1024(3)
    except (AssertionError, RuntimeError):
        return False
    return True


@pytest.mark.parametrize("mutation", [1, 2, 3, 4, 5, 6])
def test_planted_mistakes_are_caught_1024(mutation):
    assert _battery_1024()
    oracle.set_mutation(mutation)
    try:
        ok = _battery_1024()
    finally:
        oracle.set_mutation(0)
    assert not ok, f"mutation {mutation} slipped through every 1024-bit pin"
