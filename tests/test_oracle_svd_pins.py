"""Pins of the oracle's singular values (oracle.svd) against facts that do not
depend on the oracle: closed forms and exactly constructed decompositions.

* a rectangular diagonal matrix with Gaussian-integer entries of integer
  modulus (Pythagorean triples): the singular values are the moduli, exactly;
* a rank-one matrix x y^H: one singular value ||x|| ||y|| (exact here), the
  others zero;
* A = U diag(s) V^H with U, V products of phase and Hadamard matrices scaled
  to be exactly unitary (order 4 and 16, entries (+-1, +-i) / 2 or / 4) and
  dyadic s: the singular values are s, exactly;
* LAPACK (numpy) at binary64 accuracy on a seeded random rectangular matrix;
* the residual checker: zero for the exact triplets above, and it sees a
  planted error of 2^-100 in one vector entry.
A slip in the dilation (a missing conjugate, a transposed block) or in the
selection of the k largest eigenvalues (order, count) fails one of them.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle

TIGHT = 1e-60


def _fr(limbs):
    return sum((Fraction(float(x)) for x in limbs), Fraction(0))


def _hadamard_unitary(n: int, seed: int) -> np.ndarray:
    """Exactly unitary (entries (+-1, +-i) / sqrt(n), n = 4^j) phase-permuted Hadamard matrix."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H = np.array([[1.0]])
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    ph = np.array([1, 1j, -1, -1j])[rng.integers(0, 4, n)]
    perm = rng.permutation(n)
    return (ph[:, None] * H[perm]) / np.sqrt(n)


def test_rectangular_diagonal_pythagorean():
    d = [3 + 4j, -5 - 12j, 8j, 7 - 24j]          # moduli 5, 13, 8, 25
    for shape in ((6, 4), (4, 6)):
        A = np.zeros(shape, dtype=np.complex128)
        for i, z in enumerate(d):
            A[i, i] = z
        s = oracle.svd([A])
        want = sorted([5, 13, 8, 25], reverse=True)
        assert s.shape == (4, 4)
        for j in range(4):
            assert abs(_fr(s[:, j]) - want[j]) <= Fraction(TIGHT) * 25


def test_rank_one():
    x = np.array([2 + 1j, 2 - 1j, 0, 0], dtype=np.complex128)        # ||x||^2 = 10
    y = np.array([1 + 2j, 1 - 2j, 2 + 4j, 2 - 4j, 0], dtype=np.complex128)   # ||y||^2 = 50
    A = np.outer(x, y.conj())                                          # 4 x 5, s1 = sqrt(500)
    s = oracle.svd([A])
    s1 = _fr(s[:, 0])
    assert abs(s1 * s1 - 500) <= Fraction(1, 10 ** 55)
    for j in range(1, 4):
        assert abs(_fr(s[:, j])) <= Fraction(TIGHT) * 23


@pytest.mark.parametrize("n", [4, 16])
def test_exact_unitary_products(n):
    rng = np.random.Generator(np.random.PCG64(40 + n))
    svals = sorted([Fraction(int(rng.integers(1, 2 ** 20)), 2 ** int(rng.integers(0, 30))) for _ in range(n)], reverse=True)
    U = _hadamard_unitary(n, 1 + n)
    V = _hadamard_unitary(n, 2 + n)
    A = (U * np.array([float(x) for x in svals])) @ V.conj().T
    # A is exact in binary64: every entry is a dyadic sum (checked against exact rationals)
    Ue = [[(Fraction(z.real), Fraction(z.imag)) for z in row] for row in (U * np.sqrt(n)).tolist()]
    for i in range(n):
        for j in range(n):
            re = sum(svals[k] * (Ue[i][k][0] * Ve[0] + Ue[i][k][1] * Ve[1])
                     for k, Ve in ((k, (Fraction((V[j, k] * np.sqrt(n)).real), Fraction((V[j, k] * np.sqrt(n)).imag))) for k in range(n))) / n
            assert Fraction(A[i, j].real) == re
    s = oracle.svd([A])
    for j in range(n):
        assert abs(_fr(s[:, j]) - svals[j]) <= Fraction(TIGHT) * svals[0]
    # exact triplets: u_j = U e_j, v_j = V e_j have zero residual in the checker
    r, xn = oracle.svd_residuals([A], s[:2], U[None], V[None])
    assert np.all(r <= 1e-55 * float(svals[0])) and np.allclose(xn, np.sqrt(2.0))
    Vp = V.copy()
    Vp[0, 0] += 2.0 ** -100
    r2, _ = oracle.svd_residuals([A], s[:2], U[None], Vp[None])
    assert r2[0] > 1e-32 * float(svals[n - 1])


def test_lapack_rectangular():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((9, 6)) + 1j * rng.standard_normal((9, 6))
    s = oracle.svd([A])
    ref = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(s[0], ref, rtol=1e-13, atol=1e-13 * ref[0])
    sT = oracle.svd([A.conj().T])
    assert np.allclose(sT[0], ref, rtol=1e-13, atol=1e-13 * ref[0])
