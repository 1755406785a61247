"""zk_heev_mp: eigendecompositions beyond double-double (quad-double, 8 and 16
limbs) against the MPFR oracle at 1024 bits and against exact spectra.

Gates (normwise, relative to ||H||_2): eigenvalues within tol of the exact or
oracle values, every MPFR residual ||H v - lam v|| / ||v|| within tol, the
returned basis orthonormal to 100 tol; tol = 1e-60, 1e-120, 1e-240 for 4, 8,
16 limbs.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import log

pytestmark = pytest.mark.gpu

TOL = {4: 1e-60, 8: 1e-120, 16: 1e-240}
PREC = 1024


@pytest.fixture(scope="module")
def zk():
    import torch
    import paper_2402_11868_amd as Z
    Z.load()
    ctx = Z.Context(0)
    yield Z, ctx, torch
    torch.cuda.synchronize()
    ctx.close()


def _fr(limbs):
    return sum((Fraction(float(x)) for x in limbs), Fraction(0))


def _check(planes, res, ref_eigs, L, vectors=True, sample=None):
    """ref_eigs: exact Fractions or limb arrays of the ascending eigenvalues."""
    tol = TOL[L]
    w = res.w.cpu().numpy()
    n = w.shape[1]
    ref = [x if isinstance(x, Fraction) else _fr(x) for x in ref_eigs]
    hn = max(abs(x) for x in ref)
    hn = hn if hn > 0 else Fraction(1)
    err = max(abs(_fr(w[:, k]) - ref[k]) for k in range(n))
    out = {"eig": float(err / hn)}
    assert err <= Fraction(tol) * hn, f"eigenvalue error {float(err / hn):.3e} > {tol:.0e}"
    if vectors:
        V = res.V.cpu().numpy()
        idx = np.arange(n) if sample is None else np.asarray(sample)
        r, _ = oracle.residuals(planes, w[:, idx], V[:, :, idx], prec=PREC)
        out["resid"] = float(r.max() / float(hn))
        assert r.max() <= tol * float(hn), f"residual {out['resid']:.3e} > {tol:.0e}"
        mo, md = oracle.gram(V[:, :, idx], prec=PREC)
        out["orth"] = max(mo, md)
        assert mo <= 100 * tol and md <= 100 * tol, f"orthogonality {mo:.3e} / {md:.3e}"
        dev = np.array([res.info[int(k)]["resid"] for k in idx])
        out["dev_resid_max"] = float(dev.max())
    return out


@pytest.mark.parametrize("L,k", [(4, 59), (8, 200), (16, 300), (16, 700)])
@pytest.mark.parametrize("omega", [1, 1j])
def test_mp_schmidt_pair(zk, L, k, omega):
    """The paper's Schmidt pair (Sec. 1, footnote 1) with eps = 2^-k far below
    quad-double: eigenvalues exactly 1 - eps and eps."""
    Z, ctx, torch = zk
    planes, (eps, one_minus) = W.schmidt_pair(k, omega, 2)
    res, = Z.heev_mp(ctx, [[torch.from_numpy(p).cuda() for p in planes]], limbs=L)
    torch.cuda.synchronize()
    out = _check(planes, res, [eps, one_minus], L)
    log(f"mp schmidt L={L} k={k}: {out}, iterations {res.iters[0]}")
    assert res.status == Z.ZK_OK


@pytest.mark.parametrize("n,L,limbs_in,span", [(16, 8, 1, 20), (32, 16, 2, 60), (16, 16, 4, 150)])
def test_mp_hadamard_exact(zk, n, L, limbs_in, span):
    """Exact dyadic spectra with zeros and repeated eigenvalues."""
    from test_oracle_pins import _dyadic_spectrum
    Z, ctx, torch = zk
    rng = np.random.Generator(np.random.PCG64(6000 + n + L))
    lam = _dyadic_spectrum(n, rng, span, zeros=2, dups=3)
    h = W.hadamard_exact(lam, seed=33 + n, limbs=limbs_in)
    res, = Z.heev_mp(ctx, [[torch.from_numpy(p).cuda() for p in h.planes]], limbs=L)
    torch.cuda.synchronize()
    out = _check(h.planes, res, h.lam, L)
    log(f"mp hadamard n={n} L={L}: {out}, iterations {res.iters[0]}")


@pytest.mark.parametrize("n,L", [(16, 8), (40, 16), (64, 8), (64, 16)])
def test_mp_random_elements_against_1024_bit_oracle(zk, n, L):
    """Hermitian matrices with random elements (the paper's Fig. 1 workload)
    against the 1024-bit oracle, batched with a second matrix of another order."""
    Z, ctx, torch = zk
    A = W.random_elements(n, 900 + n)
    B = W.random_elements(n // 2 + 3, 901 + n)
    rs = Z.heev_mp(ctx, [[torch.from_numpy(A).cuda()], [torch.from_numpy(B).cuda()]], limbs=L)
    torch.cuda.synchronize()
    for M, r in ((A, rs[0]), (B, rs[1])):
        ref = oracle.heev([M], prec=PREC, limbs=16, want_vectors=False)
        out = _check([M], r, [ref.w_limbs[:, k] for k in range(M.shape[0])], L)
        log(f"mp random n={M.shape[0]} L={L}: {out}, iterations {r.iters[0]}")
        assert r.status == Z.ZK_OK


@pytest.mark.parametrize("n,L,k", [(24, 4, -250), (20, 8, 300), (24, 16, -200)])
def test_mp_scaled_matrices(zk, n, L, k):
    """2^k H for H with random elements: the eigenvalues are exactly 2^k times
    those of H (the 1024-bit oracle on H itself), the vectors those of H.
    Residuals at the tolerance lie far below the square root of the smallest
    binary64 here, so this also covers the range handling of the iteration.
    (k is bounded by the output format: a limb expansion of a value near 2^k
    resolves 2^(k - 1074) at best, so 1e-240 relative needs k above -270.)"""
    Z, ctx, torch = zk
    A = W.random_elements(n, 1700 + n + L)
    As = A * (2.0 ** k)
    res, = Z.heev_mp(ctx, [[torch.from_numpy(As).cuda()]], limbs=L)
    torch.cuda.synchronize()
    ref = oracle.heev([A], prec=PREC, limbs=16, want_vectors=False)
    w = res.w.cpu().numpy()
    scale = Fraction(2) ** k
    err = max(abs(_fr(w[:, j]) - _fr(ref.w_limbs[:, j]) * scale) for j in range(n))
    hn = max(abs(_fr(ref.w_limbs[:, j])) for j in range(n)) * scale
    assert err <= Fraction(TOL[L]) * hn, f"eigenvalue error {float(err / hn):.3e}"

    class Unscaled:   # the same pairs as eigenpairs of H (binary64 would underflow at 2^k tol)
        pass
    u = Unscaled()
    u.w = torch.from_numpy(w * 2.0 ** -k)
    u.V, u.info = res.V, res.info
    out = _check([A], u, [_fr(ref.w_limbs[:, j]) for j in range(n)], L)
    log(f"mp scaled 2^{k} n={n} L={L}: {out}, eigenvalue error of 2^k H {float(err / hn):.2e}, "
        f"iterations {res.iters[0]}")
    assert res.status == Z.ZK_OK


def test_mp_qd_companions(zk):
    """Quad-double through the all-pairs + polishing path on the 256 x 256
    companions of the 2048 workload: the 4-limb exact-spectrum one
    ({1 - 2^-59, 2^-59} and a geometric tail to 2^-120, exact eigenvalues) and
    the binary64-input one against the stored oracle values."""
    import golden_io as G
    Z, ctx, torch = zk
    h = W.hadamard_exact(W.spectrum_c5_dyadic(256), seed=W.seed_for(5, 100), limbs=4)
    res, = Z.heev_mp(ctx, [[torch.from_numpy(np.ascontiguousarray(p)).cuda() for p in h.planes]], limbs=4)
    torch.cuda.synchronize()
    out = _check(h.planes, res, h.lam, 4)
    log(f"mp qd exact companion: {out}, iterations {res.iters[0]}")
    assert res.status == Z.ZK_OK
    wl = W.workload(5, index=0, n=256)
    hdr, gold = G.load("c5:256:0")
    assert hdr["sha256"] == G.sha(wl["A"])
    res, = Z.heev_mp(ctx, [[torch.from_numpy(wl["A"]).cuda()]], limbs=4)
    torch.cuda.synchronize()
    out = _check([wl["A"]], res, [gold[:, k] for k in range(gold.shape[1])], 4)
    log(f"mp qd binary64-input companion: {out}, iterations {res.iters[0]}")
    assert res.status == Z.ZK_OK


def test_mp_qd_2048_whole(zk):
    """The whole 2048 x 2048 quad-double workload (4-limb exact input:
    {1 - 2^-59, 2^-59} and a geometric tail to 2^-120, the Schmidt pair of a
    60-qubit circuit, Sec. 1 footnote 1): every one of the 2048 eigenvalues
    within 1e-60 ||H||_2 of the exact spectrum, every device residual within
    the tolerance, and an MPFR sample (the pair, the largest tail values and
    the deepest ones) against their exact eigenvectors."""
    from test_gpu_workloads import _angle_sq_to_exact
    Z, ctx, torch = zk
    n = 2048
    h = W.hadamard_exact(W.spectrum_c5_dyadic(n), seed=W.seed_for(5, 0), limbs=4)
    planes = [torch.from_numpy(np.ascontiguousarray(p)).cuda() for p in h.planes]
    res, = Z.heev_mp(ctx, [planes], limbs=4)
    torch.cuda.synchronize()
    assert res.status == Z.ZK_OK
    w = res.w.cpu().numpy()
    hn = h.lam[-1]
    err = max(abs(_fr(w[:, k]) - h.lam[k]) for k in range(n))
    assert err <= Fraction(TOL[4]) * hn, f"eigenvalue error {float(err / hn):.3e}"
    dev = max(x["resid"] for x in res.info)
    assert dev <= TOL[4], f"device residual {dev:.3e}"
    sample = np.array(list(range(0, 16)) + [n // 2] + list(range(n - 18, n)))
    V = res.V.cpu().numpy()
    r, _ = oracle.residuals(h.planes, w[:, sample], V[:, :, sample])
    assert r.max() <= TOL[4] * float(hn)
    E = h.vectors_unnormalised()
    worst = Fraction(0)
    lam = h.lam
    for k in sample:
        # eigenvectors are unique here (no repeated eigenvalue); the bound is
        # Davis-Kahan: sin(angle) <= residual / gap, residual <= tol ||H||_2
        k = int(k)
        gap = min(abs(lam[k] - lam[j]) for j in (k - 1, k + 1) if 0 <= j < n)
        s2 = _angle_sq_to_exact(V, k, E[:, k])
        bound = (Fraction(TOL[4]) * hn / gap) ** 2
        assert s2 <= bound, f"pair {k}: sin^2(angle) {float(s2):.3e} above {float(bound):.3e}"
        worst = max(worst, s2 / bound)
    log(f"mp qd 2048: eigenvalue error {float(err / hn):.2e}, device residual {dev:.2e}, MPFR residual (sample) "
        f"{r.max() / float(hn):.2e}, sin^2 angle / Davis-Kahan bound (sample) {float(worst):.2e}, "
        f"iterations {res.iters[0]}")


def test_mp_errors(zk):
    Z, ctx, torch = zk
    A = torch.from_numpy(W.random_elements(8, 1)).cuda()
    for L in (2, 5):
        with pytest.raises(RuntimeError, match="ZK_EINVAL"):
            Z.heev_mp(ctx, [[A]], limbs=L)
