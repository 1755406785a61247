"""The MPS simulation driver (zk_mps_*): two-qubit gates turn into Hermitian
bond matrices eigendecomposed through a serving session.

* The paper's introductory state, C^(n-1)-Z on |+>^(n-1) |-> (Sec. 1, footnote
  1), prepared from |0...0> by a nearest-neighbour staircase of two-qubit
  gates at 24, 40 and 60 qubits: every bond keeps dimension 2 and its squared
  Schmidt values match the closed form (eigenvalues of the 2 x 2 product of
  the branches' Gram matrices, in mpmath) within 1e-30; across the last cut
  they are exactly 1 - eps and eps with eps = 2^-(n-1).
* An 8-qubit brickwork of dyadic unitary gates: the contracted MPS equals the
  exact rational state vector (oracle.apply_gate) within 1e-29 in every
  amplitude; every bond matrix went through the session.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
import workloads as W

from gpu_helpers import log
from test_gpu_mps import GATES, _fr, _fr_gate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zk():
    import torch
    import paper_2402_11868_amd as Z
    Z.load()
    ctx = Z.Context(0)
    yield Z, ctx, torch
    torch.cuda.synchronize()
    ctx.close()


def _cnz_bond_spectrum(n, b):
    """Exact squared Schmidt values (descending) of the C^(n-1)-Z state across
    the cut after b qubits: psi = |L_a>|R_a> + |L_b>|R_b> with L_a = |+>^b,
    L_b = |1>^b, R_a = |+>^(n-1-b) |->, R_b = c |1>^(n-b), c = 2^-((n-2)/2)."""
    mpmath.mp.dps = 80
    c = mpmath.mpf(2) ** (-mpmath.mpf(n - 2) / 2)
    gl = mpmath.mpf(2) ** (-mpmath.mpf(b) / 2)                      # <L_a|L_b>
    gr = -c * mpmath.mpf(2) ** (-mpmath.mpf(n - b) / 2)            # <R_a|R_b>
    GL = mpmath.matrix([[1, gl], [gl, 1]])
    GR = mpmath.matrix([[1, gr], [gr, c * c]])                     # <R_i|R_j>
    M = GR.T * GL
    tr = M[0, 0] + M[1, 1]
    det = M[0, 0] * M[1, 1] - M[0, 1] * M[1, 0]
    disc = mpmath.sqrt(tr * tr - 4 * det)
    return [(tr + disc) / 2, (tr - disc) / 2]


@pytest.mark.parametrize("n", [24, 40, 60])
def test_mps_sim_cnz_state(zk, n):
    Z, ctx, torch = zk
    m = Z.Mps(ctx, n, chi_max=8, cutoff=1e-14)
    for k, hi, lo in W.cnz_staircase(n):
        assert m.apply2([k], [(hi, lo)]) == Z.ZK_OK
    worst = mpmath.mpf(0)
    mpmath.mp.dps = 80
    for b in range(1, n):
        e = m.bond(b)
        assert e.shape[1] == 2, f"bond {b}: dimension {e.shape[1]}"
        ref = _cnz_bond_spectrum(n, b)
        for j in range(2):
            got = mpmath.mpf(float(e[0, j])) + mpmath.mpf(float(e[1, j]))
            worst = max(worst, abs(got - ref[j]))
    assert worst <= mpmath.mpf("1e-30"), f"bond spectra off by {float(worst):.3e}"
    e = m.bond(n - 1)
    eps = Fraction(1, 2 ** (n - 1))
    got_eps = _fr(e[:, 1])
    got_one = _fr(e[:, 0])
    assert abs(got_eps - eps) <= Fraction(1, 10 ** 30) and abs(got_one - (1 - eps)) <= Fraction(1, 10 ** 30)
    lat, orders = m.latencies()
    assert len(lat) == n - 1
    log(f"mps sim C^(n-1)-Z n={n}: worst bond-spectrum error {float(worst):.2e}, last cut eps rel. error "
        f"{float(abs(got_eps - eps) / eps):.2e}, bond matrices {len(lat)}, p50 latency {1e3 * np.median(lat):.2f} ms")
    m.close()


def test_mps_sim_brickwork_exact(zk):
    Z, ctx, torch = zk
    n = 8
    m = Z.Mps(ctx, n, chi_max=16, cutoff=1e-14)
    psi = [(Fraction(0), Fraction(0))] * (2 ** n)
    psi[0] = (Fraction(1), Fraction(0))
    count = 0
    for layer in range(6):
        qs = list(range(0, n - 1, 2) if layer % 2 == 0 else range(1, n - 1, 2))
        gs = [GATES[(3 * layer + q) % len(GATES)] for q in qs]
        assert m.apply2(qs, gs) == Z.ZK_OK
        count += len(qs)
        for q, G in zip(qs, gs):
            psi = oracle.apply_gate(psi, n, q, _fr_gate(G))
    sites = [m.site(q) for q in range(n)]
    mats = []
    for h in sites:
        cl, cr = h.shape[1], h.shape[3]
        mats.append([[[(_fr([h[0, a, p, b].real, h[1, a, p, b].real]), _fr([h[0, a, p, b].imag, h[1, a, p, b].imag]))
                       for b in range(cr)] for a in range(cl)] for p in range(2)])
    worst = Fraction(0)
    for x in range(2 ** n):
        bits = [(x >> (n - 1 - k)) & 1 for k in range(n)]
        vec = [(Fraction(1), Fraction(0))]
        for k in range(n):
            Mk = mats[k][bits[k]]
            vec = [(sum((vec[a][0] * Mk[a][b][0] - vec[a][1] * Mk[a][b][1] for a in range(len(vec))), Fraction(0)),
                    sum((vec[a][0] * Mk[a][b][1] + vec[a][1] * Mk[a][b][0] for a in range(len(vec))), Fraction(0)))
                   for b in range(len(Mk[0]))]
        worst = max(worst, abs(vec[0][0] - psi[x][0]), abs(vec[0][1] - psi[x][1]))
    assert worst <= Fraction(1, 10 ** 29), f"amplitude error {float(worst):.3e}"
    lat, orders = m.latencies()
    assert len(lat) == count
    log(f"mps sim brickwork n={n}: bond dimensions {[s.shape[1] for s in sites[1:]]}, max amplitude error "
        f"{float(worst):.2e}, {count} bond matrices of orders {sorted(set(orders.tolist()))}")
    m.close()


def test_mps_sim_errors(zk):
    Z, ctx, torch = zk
    m = Z.Mps(ctx, 6, chi_max=4)
    G = np.eye(4, dtype=np.complex128)
    with pytest.raises(RuntimeError, match="ZK_EINVAL"):
        m.apply2([0, 1], [G, G])          # overlapping pairs
    with pytest.raises(RuntimeError, match="ZK_EINVAL"):
        m.apply2([5], [G])                # no qubit 6
    with pytest.raises(RuntimeError, match="ZK_EINVAL"):
        Z.Mps(ctx, 1)
    m.close()
