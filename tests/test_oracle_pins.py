"""Pins of the MPFR oracle against facts that do not depend on the oracle itself.

Each pin is chosen so that a plausible slip in the Jacobi solver (a dropped
conjugate, a wrong rotation sign, a dropped phase, a transposed read, vectors
not accumulated, a limb ignored) fails at least one of them; the last test
plants each of those slips in the oracle and checks exactly that.

Pins:
* the paper's Schmidt pair (Sec. 1, footnote 1): eigenvalues exactly 1-eps and
  eps with eps = 2^-k, eigenvectors (1, +-conj(w))/sqrt 2;
* exact-spectrum Hadamard matrices: eigenvalues and eigenspaces known exactly;
* n <= 4: roots of the exact rational characteristic polynomial (mpmath);
* invariants trace(H) = sum(lam), ||H||_F^2 = sum(lam^2) in exact rationals;
* mpmath.eighe at 80 digits and LAPACK (numpy) at binary64 accuracy.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
import workloads as W

TIGHT = 1e-62  # 4-limb (~2^-212 relative) output resolution of the 256-bit oracle


def _frac_sum(limbs):
    return sum((Fraction(float(x)) for x in limbs), Fraction(0))


def _eig_fracs(res):
    return [_frac_sum(res.w_limbs[:, k]) for k in range(res.w_limbs.shape[1])]


def _vec(res, k, limbs=4):
    """Eigenvector k as an mpmath vector (exact limb sum)."""
    n = res.v_limbs.shape[1]
    out = []
    for i in range(n):
        re = sum(mpmath.mpf(float(res.v_limbs[l, i, k].real)) for l in range(limbs))
        im = sum(mpmath.mpf(float(res.v_limbs[l, i, k].imag)) for l in range(limbs))
        out.append(mpmath.mpc(re, im))
    return out


# ------------------------------------------------------------------ pins --

@pytest.mark.parametrize("k,limbs", [(2, 1), (10, 1), (39, 1), (53, 1), (59, 2), (100, 2), (150, 4)])
@pytest.mark.parametrize("omega", [1, -1, 1j, -1j])
def test_schmidt_pair_exact(k, limbs, omega):
    planes, (eps, one_minus) = W.schmidt_pair(k, omega, limbs)
    r = oracle.heev(planes)
    lam = _eig_fracs(r)
    assert abs(lam[0] - eps) <= Fraction(1, 2 ** 205)
    assert abs(lam[1] - one_minus) <= Fraction(1, 2 ** 205)
    mpmath.mp.dps = 90
    # v_{1-eps} = (1, conj w)/sqrt2 ; v_eps = (1, -conj w)/sqrt2
    w = mpmath.mpc(complex(omega).real, complex(omega).imag)
    for idx, sgn in ((1, 1), (0, -1)):
        v = _vec(r, idx)
        ex = [1 / mpmath.sqrt(2), sgn * mpmath.conj(w) / mpmath.sqrt(2)]
        ov = abs(mpmath.conj(ex[0]) * v[0] + mpmath.conj(ex[1]) * v[1])
        assert abs(ov - 1) < 1e-60


def _dyadic_spectrum(n, rng, span_bits, mant_bits=12, zeros=0, dups=0):
    vals = []
    for _ in range(n - zeros - dups):
        e = int(rng.integers(0, span_bits))
        m = int(rng.integers(1, 2 ** mant_bits))
        vals.append(Fraction(m, 2 ** (mant_bits + e)))
    for j in range(dups):
        vals.append(vals[j])
    vals += [Fraction(0)] * zeros
    return vals


@pytest.mark.parametrize("n,limbs,span", [(16, 1, 20), (32, 1, 24), (64, 2, 60), (16, 4, 150)])
def test_hadamard_exact_spectrum_and_spaces(n, limbs, span):
    rng = np.random.Generator(np.random.PCG64(1000 + n + limbs))
    lam = _dyadic_spectrum(n, rng, span, zeros=2, dups=3)
    h = W.hadamard_exact(lam, seed=77 + n, limbs=limbs)
    r = oracle.heev(h.planes)
    got = _eig_fracs(r)
    scale = max(abs(x) for x in lam)
    for a, b in zip(got, h.lam):
        assert abs(a - b) <= scale * Fraction(1, 2 ** 205)
    # eigenspaces: every oracle vector of eigenvalue mu lies in the exact eigenspace of mu
    Vx = h.vectors_unnormalised() / np.sqrt(n)
    V = r.v_limbs[0] + r.v_limbs[1]
    distinct = sorted(set(h.lam))
    for mu in distinct:
        idx = [i for i, x in enumerate(h.lam) if x == mu]
        Q = Vx[:, idx]
        P = V[:, idx]
        resid = P - Q @ (Q.conj().T @ P)
        assert np.abs(resid).max() < 1e-13  # binary64 evaluation of an exact-zero projection
        assert np.abs(P.conj().T @ P - np.eye(len(idx))).max() < 1e-13


def _charpoly_exact(H):
    """det(xI - H) coefficients (highest first) by Faddeev-LeVerrier in exact Gaussian rationals."""
    n = H.shape[0]
    A = [[(Fraction(float(H[i, j].real)), Fraction(float(H[i, j].imag))) for j in range(n)] for i in range(n)]
    # enforce the lower-triangle convention: upper = conj(lower), real diagonal
    for i in range(n):
        A[i][i] = (A[i][i][0], Fraction(0))
        for j in range(i + 1, n):
            A[i][j] = (A[j][i][0], -A[j][i][1])

    def mul(X, Y):
        Z = [[(Fraction(0), Fraction(0))] * n for _ in range(n)]
        for i in range(n):
            for j in range(n):
                re = Fraction(0)
                im = Fraction(0)
                for k in range(n):
                    a, b = X[i][k], Y[k][j]
                    re += a[0] * b[0] - a[1] * b[1]
                    im += a[0] * b[1] + a[1] * b[0]
                Z[i][j] = (re, im)
        return Z

    c = [Fraction(1)]
    M = [[(Fraction(0), Fraction(0))] * n for _ in range(n)]
    for k in range(1, n + 1):
        M = [[(M[i][j][0] + (c[-1] if i == j else 0), M[i][j][1]) for j in range(n)] for i in range(n)]
        AM = mul(A, M)
        tr_re = sum(AM[i][i][0] for i in range(n))
        tr_im = sum(AM[i][i][1] for i in range(n))
        assert tr_im == 0
        c.append(-tr_re / k)
        M = AM
    return c


@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("seed", [11, 12])
def test_small_n_charpoly_roots(n, seed):
    A = W.random_elements(n, seed)
    r = oracle.heev([A])
    coeffs = _charpoly_exact(A)
    mpmath.mp.dps = 100
    roots = sorted(mpmath.re(z) for z in mpmath.polyroots([mpmath.mpf(x.numerator) / x.denominator for x in coeffs],
                                                          maxsteps=400, extraprec=400))
    got = _eig_fracs(r)
    for a, b in zip(got, roots):
        assert abs(mpmath.mpf(a.numerator) / a.denominator - b) < TIGHT


def test_n2_closed_form():
    A = W.random_elements(2, 5)
    a, d = A[0, 0].real, A[1, 1].real
    b = A[1, 0]
    mpmath.mp.dps = 100
    m = (mpmath.mpf(a) + mpmath.mpf(d)) / 2
    rad = mpmath.sqrt(((mpmath.mpf(a) - mpmath.mpf(d)) / 2) ** 2 + mpmath.mpf(b.real) ** 2 + mpmath.mpf(b.imag) ** 2)
    r = oracle.heev([A])
    got = _eig_fracs(r)
    for g, ex in zip(got, (m - rad, m + rad)):
        assert abs(mpmath.mpf(g.numerator) / g.denominator - ex) < TIGHT


@pytest.mark.parametrize("n", [17, 48])
def test_trace_and_frobenius_invariants(n):
    lam = W.spectrum_c4(n)
    A = W.householder_hermitian(lam, seed=W.seed_for(4, n))
    r = oracle.heev([A], want_vectors=False)
    got = _eig_fracs(r)
    tr = sum(Fraction(float(A[i, i].real)) for i in range(n))
    fro = Fraction(0)
    for i in range(n):
        for j in range(n):
            z = A[i, j] if i >= j else np.conj(A[j, i])
            re = Fraction(float(z.real))
            im = Fraction(0) if i == j else Fraction(float(z.imag))
            fro += re * re + im * im
    assert abs(sum(got) - tr) < Fraction(1, 10 ** 60)
    assert abs(sum(x * x for x in got) - fro) < Fraction(1, 10 ** 60)


def test_mpmath_eighe_n10():
    A = W.random_elements(10, 3)
    mpmath.mp.dps = 80
    M = mpmath.matrix(10, 10)
    for i in range(10):
        for j in range(10):
            z = A[i, j] if i >= j else np.conj(A[j, i])
            M[i, j] = mpmath.mpc(float(z.real), 0.0 if i == j else float(z.imag))
    E, _ = mpmath.eighe(M)
    ev = sorted(E[i] for i in range(10))
    r = oracle.heev([A], want_vectors=False)
    got = _eig_fracs(r)
    for g, e in zip(got, ev):
        assert abs(mpmath.mpf(g.numerator) / g.denominator - e) < TIGHT


def test_lapack_agreement_n100():
    A = W.random_elements(100, 9)
    r = oracle.heev([A], want_vectors=False)
    ev = np.linalg.eigvalsh(A)
    nrm = np.abs(ev).max()
    assert np.abs(r.w - ev).max() <= 100 * 100 * 2.0 ** -53 * nrm


# ------------------------------------------------------------- checkers --

def test_residual_and_gram_checkers_exact_and_perturbed():
    lam = [Fraction(k, 8) for k in range(16)]
    h = W.hadamard_exact(lam, seed=3, limbs=1)
    V = h.vectors_unnormalised() / 4.0  # exact: n = 16, sqrt(n) = 4
    w = np.array([float(x) for x in h.lam])
    res, vn = oracle.residuals(h.planes, w[None], V[None])
    assert res.max() == 0.0 and np.all(vn == 1.0)
    mo, md = oracle.gram(V[None])
    assert mo == 0.0 and md == 0.0
    # perturb one component of vector 5 by delta (second limb): residual = |delta| ||(H - lam I) e_i|| / ||v||
    delta = 2.0 ** -80
    V2 = np.zeros_like(V)
    V2[3, 5] = delta
    res, vn = oracle.residuals(h.planes, w[None], np.stack([V, V2]))
    H = h.planes[0]
    col = H[:, 3].copy()
    col[3] -= w[5]
    expect = delta * np.linalg.norm(col) / np.sqrt(1.0 + 2 * delta * V[3, 5].real + delta ** 2)
    assert abs(res[5] - expect) <= 1e-12 * expect
    assert np.all(res[np.arange(16) != 5] == 0.0)
    mo, md = oracle.gram(np.stack([V, V2]))
    # |v_j^H v_5| for j != 5 is delta |V[3, j]| = delta/4 ; diag: |2 delta Re V[3,5] + delta^2|
    assert abs(mo - delta / 4) <= 1e-12 * delta
    assert abs(md - abs(2 * delta * V[3, 5].real + delta ** 2)) <= 1e-12 * delta


# ------------------------------------------------------------ mutations --

def _battery():
    """Quick pins; returns True if all pass."""
    try:
        test_schmidt_pair_exact(59, 2, 1j)
        test_hadamard_exact_spectrum_and_spaces(16, 1, 20)
        test_small_n_charpoly_roots(3, 11)
    except (AssertionError, RuntimeError):
        return False
    return True


@pytest.mark.parametrize("mutation", [1, 2, 3, 4, 5, 6])
def test_planted_mistakes_are_caught(mutation):
    assert _battery()
    oracle.set_mutation(mutation)
    try:
        ok = _battery()
    finally:
        oracle.set_mutation(0)
    assert not ok, f"mutation {mutation} slipped through every pin"
