"""The double-double MPS two-site update (zk_mps_two_site_dd) against exact
rational references (oracle.two_site_theta, oracle.apply_gate) and the MPFR
SVD, under both refinements.

* One update (chi_l 8, chi 12, chi_r 10): singular values within 1e-30 s_1 of
  the oracle's SVD of the exact theta' = G (A B); A' B' reproduces theta'
  within 4e-30 s_1 and A' has orthonormal columns (1e-28); a cut to chi' = 6
  keeps the 6 largest values and leaves the Eckart-Young error
  sum_{j >= 6} s_j^2.
* A 6-qubit chain from |000000> through 5 brickwork layers of dyadic unitary
  two-qubit gates (products of (1/2) Sylvester = H x H, CNOT, CZ and
  diag(1, i, -1, -i), exact in binary64), every gate one two-site update with
  singular values below 1e-28 s_1 dropped: the contracted MPS equals the
  exact rational state vector within 1e-29 in every amplitude.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle

from gpu_helpers import log

pytestmark = pytest.mark.gpu

TOL, ORTH = 1e-30, 1e-28


@pytest.fixture(scope="module")
def zk():
    import torch
    import paper_2402_11868_amd as Z
    Z.load()
    ctx = Z.Context(0)
    yield Z, ctx, torch
    torch.cuda.synchronize()
    ctx.close()


W = 0.5 * np.array([[1, 1, 1, 1], [1, -1, 1, -1], [1, 1, -1, -1], [1, -1, -1, 1]], dtype=np.complex128)
CNOT = np.eye(4, dtype=np.complex128)[[0, 1, 3, 2]]
CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)
PH = np.diag([1, 1j, -1, -1j]).astype(np.complex128)
GATES = [CNOT @ W, CZ @ W, PH @ CNOT @ W, W @ CZ @ PH]


def _fr_gate(G):
    return [[(Fraction(float(G[i, j].real)), Fraction(float(G[i, j].imag))) for j in range(4)] for i in range(4)]


def _fr(limbs):
    return sum((Fraction(float(x)) for x in limbs), Fraction(0))


def _cfr(planes, i, j):
    return (_fr([p[i, j].real for p in planes]), _fr([p[i, j].imag for p in planes]))


@pytest.mark.parametrize("refine", [0, 1])
def test_two_site_update_against_oracle(zk, refine):
    Z, ctx, torch = zk
    cl, chi, cr = 8, 12, 10
    M, N = 2 * cl, 2 * cr
    rng = np.random.default_rng(2024)
    A = rng.standard_normal((M, chi)) + 1j * rng.standard_normal((M, chi))
    B = rng.standard_normal((chi, N)) + 1j * rng.standard_normal((chi, N))
    G = GATES[0]
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    r = Z.mps_two_site(ctx, dev(A), dev(B), dev(G), chi_max=min(M, N), opts=Z.make_opts(refine=refine))
    assert r.status == Z.ZK_OK and r.chi == min(M, N)
    T = oracle.two_site_theta([A], [B], _fr_gate(G))
    ref = oracle.svd(oracle.limb_planes(T, 4))
    s = r.s.cpu().numpy()
    ref_s = [_fr(ref[:, j]) for j in range(r.chi)]
    s1 = ref_s[0]
    err = max(abs(_fr(s[:, j]) - ref_s[j]) for j in range(r.chi))
    assert err <= Fraction(TOL) * s1, f"singular values off by {float(err / s1):.3e} s_1"
    Ap = [x for x in r.A.cpu().numpy()]
    Bp = [x for x in r.B.cpu().numpy()]
    worst = Fraction(0)
    for i in range(M):
        for j in range(N):
            re, im = Fraction(0), Fraction(0)
            for k in range(r.chi):
                a = _cfr(Ap, i, k)
                b = _cfr(Bp, k, j)
                re += a[0] * b[0] - a[1] * b[1]
                im += a[0] * b[1] + a[1] * b[0]
            worst = max(worst, abs(re - T[i][j][0]), abs(im - T[i][j][1]))
    assert worst <= 4 * Fraction(TOL) * s1, f"A' B' off theta' by {float(worst / s1):.3e} s_1"
    mo, md = oracle.gram(r.A.cpu().numpy())
    assert mo <= ORTH and md <= ORTH
    cut = Z.mps_two_site(ctx, dev(A), dev(B), dev(G), chi_max=6, opts=Z.make_opts(refine=refine))
    assert cut.chi == 6
    sc = cut.s.cpu().numpy()
    assert max(abs(_fr(sc[:, j]) - ref_s[j]) for j in range(6)) <= Fraction(TOL) * s1
    Ac = [x for x in cut.A.cpu().numpy()]
    Bc = [x for x in cut.B.cpu().numpy()]
    resid2 = Fraction(0)
    for i in range(M):
        for j in range(N):
            re, im = T[i][j]
            for k in range(6):
                a = _cfr(Ac, i, k)
                b = _cfr(Bc, k, j)
                re -= a[0] * b[0] - a[1] * b[1]
                im -= a[0] * b[1] + a[1] * b[0]
            resid2 += re * re + im * im
    tail = sum((x * x for x in ref_s[6:]), Fraction(0))
    assert abs(resid2 - tail) <= Fraction(1, 10 ** 28) * s1 * s1
    log(f"two-site update refine={refine}: s err {float(err / s1):.2e}, reconstruction {float(worst / s1):.2e}")


@pytest.mark.parametrize("refine", [0, 1])
def test_mps_circuit_against_exact_state(zk, refine):
    """Clifford gates give two-site matrices with equal singular values and
    exact zeros: dilations whose tridiagonal splits into blocks sharing an
    eigenvalue (the inverse iteration takes negligible couplings as zeros)."""
    Z, ctx, torch = zk
    n = 6
    sites = []
    for _ in range(n):
        t = torch.zeros((2, 1, 2, 1), dtype=torch.complex128, device="cuda")
        t[0, 0, 0, 0] = 1.0
        sites.append(t)
    psi = [(Fraction(0), Fraction(0))] * (2 ** n)
    psi[0] = (Fraction(1), Fraction(0))
    chis = []
    for layer in range(5):
        for q in (range(0, n - 1, 2) if layer % 2 == 0 else range(1, n - 1, 2)):
            G = GATES[(3 * layer + q) % len(GATES)]
            Tl, Tr = sites[q], sites[q + 1]
            cl, cm, cr = Tl.shape[1], Tl.shape[3], Tr.shape[3]
            A = [Tl[l].permute(1, 0, 2).reshape(2 * cl, cm) for l in range(2)]
            B = [Tr[l].reshape(cm, 2 * cr) for l in range(2)]
            r = Z.mps_two_site(ctx, A, B, torch.from_numpy(G).cuda(), chi_max=min(2 * cl, 2 * cr), cutoff=1e-28,
                               opts=Z.make_opts(refine=refine))
            assert r.status == Z.ZK_OK
            c = r.chi
            sites[q] = torch.stack([r.A[l].reshape(2, cl, c).permute(1, 0, 2) for l in range(2)]).contiguous()
            sites[q + 1] = torch.stack([r.B[l].reshape(c, 2, cr) for l in range(2)]).contiguous()
            psi = oracle.apply_gate(psi, n, q, _fr_gate(G))
        chis.append([int(s.shape[3]) for s in sites[:-1]])
    torch.cuda.synchronize()
    # contract the chain exactly from the returned limbs
    mats = []
    for s in sites:
        h = s.cpu().numpy()
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
    log(f"mps circuit n={n} refine={refine}: bond dimensions per layer {chis}, max amplitude error {float(worst):.2e}")


def test_two_site_update_errors(zk):
    """Argument errors are rejected before any device work (ZK_EINVAL, raised by
    the binding as RuntimeError; shape mismatches as ValueError)."""
    Z, ctx, torch = zk
    A = torch.zeros((4, 3), dtype=torch.complex128, device="cuda")
    B = torch.zeros((3, 6), dtype=torch.complex128, device="cuda")
    G = torch.eye(4, dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError):
        Z.mps_two_site(ctx, A, B, G, chi_max=0)
    with pytest.raises(RuntimeError):
        Z.mps_two_site(ctx, A, B, G, chi_max=5)       # above min(2 chi_l, 2 chi_r) = 4
    with pytest.raises(RuntimeError):
        Z.mps_two_site(ctx, A, B, G, chi_max=2, cutoff=float("nan"))
    with pytest.raises(ValueError):
        Z.mps_two_site(ctx, A, torch.zeros((2, 6), dtype=torch.complex128, device="cuda"), G, chi_max=2)
    r = Z.mps_two_site(ctx, A, B, G, chi_max=2)          # the zero state: chi' = 1, s = 0
    assert r.status == Z.ZK_OK and r.chi == 1
    assert float(r.s[0, 0]) == 0.0
