"""The blocking scheme of the LDL^H shifted solves (tests/ldl_model.py, the
GPU kernels' steps and slot layout in binary64) against numpy's solver:
backward error at binary64 level on indefinite, 2x2-heavy (zero diagonal),
graded and designed-spectrum matrices shifted onto their eigenvalues, with
look-ahead windows of 1, 2 and 4 columns; the counts show that the
interchange paths (inside and outside the window), 2x2 blocks and panels
that end one column early before a 2x2 block were all taken."""
import numpy as np
import pytest

import ldl_model as model
import workloads as W


def _backward(A, x, b):
    return np.linalg.norm(A @ x - b) / (np.linalg.norm(A, 2) * np.linalg.norm(x) + np.linalg.norm(b))


def _cases(n, rng):
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    yield "random", (Z + Z.conj().T) / 2
    m = n // 2
    Bm = rng.standard_normal((m, n - m)) + 1j * rng.standard_normal((m, n - m))
    A = np.zeros((n, n), complex)
    A[:m, m:] = Bm
    A[m:, :m] = Bm.conj().T
    yield "zero diagonal", A
    A = W.householder_hermitian(W.spectrum_c4(n), seed=W.seed_for(4, n))
    yield "designed spectrum", np.tril(A) + np.tril(A, -1).conj().T


@pytest.mark.parametrize("la", [1, 2, 4])
def test_blocked_ldl_backward_error(la):
    rng = np.random.default_rng(2024 + la)
    tot = {}
    worst = 0.0
    for n in (33, 75):
        for name, A in _cases(n, rng):
            w = np.linalg.eigvalsh(A)
            for sig in (w[n // 3] * (1 + 1e-9), w[-1] * (1 - 1e-12), 0.0):
                B = A - sig * np.eye(n)
                b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
                x, st = model.solve(B, b, 1e-18 * np.abs(w).max(), None, la)
                for k, v in st.items():
                    tot[k] = tot.get(k, 0) + v
                r = _backward(B, x, b)
                worst = max(worst, r)
                assert r <= 1e-14, f"{name} n={n} sigma={sig:.3e}: backward error {r:.2e}"
    assert tot["swap"] > 0 and tot["2x2"] > 0 and tot.get("short_panels", 0) > 0, tot
    if la > 1:
        assert tot["kp_in"] > 0, tot
