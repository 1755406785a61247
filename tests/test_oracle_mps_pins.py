"""Pins of the oracle's exact MPS references (oracle.two_site_theta,
oracle.apply_gate, oracle.limb_planes) against facts that do not depend on
them: closed-form states, exact unitary invariance, inverse gates, and a CNOT
chain that must map |100000> to |111111> (site 0 most significant)."""
from fractions import Fraction

import numpy as np

import oracle

F0, F1, FH = Fraction(0), Fraction(1), Fraction(1, 2)


def cnot():
    perm = [0, 1, 3, 2]
    return [[(F1 if perm[i] == j else F0, F0) for j in range(4)] for i in range(4)]


def sylvester_half():
    S = [[1, 1, 1, 1], [1, -1, 1, -1], [1, 1, -1, -1], [1, -1, -1, 1]]
    return [[(FH * S[i][j], F0) for j in range(4)] for i in range(4)]


def adjoint(G):
    return [[(G[j][i][0], -G[j][i][1]) for j in range(4)] for i in range(4)]


def test_bell_state_from_cnot():
    # |+>|0> unnormalised: A = [1, 1]^T (s1), B = [1, 0] (s2); CNOT -> |00> + |11>
    A = [np.array([[1.0], [1.0]], dtype=np.complex128)]
    B = [np.array([[1.0, 0.0]], dtype=np.complex128)]
    T = oracle.two_site_theta(A, B, cnot())
    assert [[T[i][j][0] for j in range(2)] for i in range(2)] == [[1, 0], [0, 1]]
    assert all(T[i][j][1] == 0 for i in range(2) for j in range(2))


def test_unitary_gate_keeps_the_norm_exactly():
    rng = np.random.default_rng(3)
    A = [rng.standard_normal((6, 4)) + 1j * rng.standard_normal((6, 4))]
    B = [rng.standard_normal((4, 8)) + 1j * rng.standard_normal((4, 8))]
    I = [[(F1 if i == j else F0, F0) for j in range(4)] for i in range(4)]
    T0 = oracle.two_site_theta(A, B, I)
    T1 = oracle.two_site_theta(A, B, sylvester_half())
    nrm = lambda T: sum(x[0] ** 2 + x[1] ** 2 for row in T for x in row)
    assert nrm(T0) == nrm(T1)


def test_gate_then_adjoint_is_identity_and_cnot_chain():
    n = 6
    rng = np.random.default_rng(4)
    psi = [(Fraction(int(rng.integers(-9, 10)), 16), Fraction(int(rng.integers(-9, 10)), 16)) for _ in range(2 ** n)]
    G = sylvester_half()
    out = oracle.apply_gate(oracle.apply_gate(psi, n, 2, G), n, 2, adjoint(G))
    assert out == psi
    basis = [(F0, F0)] * (2 ** n)
    basis[1 << (n - 1)] = (F1, F0)
    for q in range(n - 1):
        basis = oracle.apply_gate(basis, n, q, cnot())
    assert basis[2 ** n - 1] == (F1, F0)
    assert sum(1 for x in basis if x != (F0, F0)) == 1


def test_limb_planes_split():
    T = [[(Fraction(1, 3), Fraction(-2, 7))]]
    P = oracle.limb_planes(T, L=4)
    assert P[0][0, 0] == complex(1 / 3, -2 / 7)
    re = sum((Fraction(float(p[0, 0].real)) for p in P), Fraction(0))
    im = sum((Fraction(float(p[0, 0].imag)) for p in P), Fraction(0))
    assert abs(re - Fraction(1, 3)) < Fraction(1, 2 ** 210)
    assert abs(im + Fraction(2, 7)) < Fraction(1, 2 ** 210)


def test_limb_sum_matrix_two_and_four_planes():
    """limb_sum_matrix on more than one plane: values that binary64 cannot
    hold (1 + 2^-60, -3 + 2^-70 i, a four-limb 2^-200 tail, limbs of opposite
    signs that cancel) must come back exactly, in both the real and the
    imaginary part and at every position of a non-square matrix."""
    P0 = np.array([[1.0, 1j * -3.0, 2.0 ** 40], [0.25j, -1.0, 0.0]], dtype=np.complex128)
    P1 = np.array([[2.0 ** -60, 1j * 2.0 ** -70, -1.0], [2.0 ** -80, 2.0 ** -53 * 1j, -(2.0 ** -90)]], dtype=np.complex128)
    S = oracle.limb_sum_matrix([P0, P1])
    assert len(S) == 2 and len(S[0]) == 3
    assert S[0][0] == (1 + Fraction(1, 2 ** 60), F0)
    assert S[0][1] == (F0, -3 + Fraction(1, 2 ** 70))
    assert S[0][2] == (Fraction(2 ** 40 - 1), F0)
    assert S[1][0] == (Fraction(1, 2 ** 80), Fraction(1, 4))
    assert S[1][1] == (Fraction(-1), Fraction(1, 2 ** 53))
    assert S[1][2] == (-Fraction(1, 2 ** 90), F0)
    # four planes: 1 + 2^-60 + 2^-130 i + 2^-200, and a full cancellation
    Q = [np.array([[1.0, 1.0]]), np.array([[2.0 ** -60, -1.0]]), np.array([[2.0 ** -130 * 1j, 0.0]]),
         np.array([[2.0 ** -200, 0.0]])]
    S4 = oracle.limb_sum_matrix([q.astype(np.complex128) for q in Q])
    assert S4[0][0] == (1 + Fraction(1, 2 ** 60) + Fraction(1, 2 ** 200), Fraction(1, 2 ** 130))
    assert S4[0][1] == (F0, F0)
    # round trip through the greedy split of exact dyadic values needing four limbs
    rng = np.random.default_rng(9)
    T = [[(Fraction(int(rng.integers(-2 ** 40, 2 ** 40)), 1) + Fraction(int(rng.integers(1, 2 ** 40)), 2 ** 150),
           Fraction(int(rng.integers(-2 ** 40, 2 ** 40)), 2 ** 100)) for _ in range(3)] for _ in range(2)]
    assert oracle.limb_sum_matrix(oracle.limb_planes(T, L=4)) == T
