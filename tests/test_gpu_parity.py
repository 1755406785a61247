"""Parity of the HIP path (through the C-ABI) with the MPFR oracle.

Bar (the accuracy the workloads are specified with; the paper fixes no
tolerance): eigenvalue error and residual
||H v - lam v|| / ||v|| both <= 1e-30 ||H||_2 for double-double output and
<= 1e-60 ||H||_2 for quad-double output; orthogonality max |v_i^H v_j| <=
1e-28 (dd) / 1e-58 (qd).  Every check is evaluated on the returned limbs
exactly as returned.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W

from gpu_helpers import gate, log, to_np

pytestmark = pytest.mark.gpu

DD_TOL, QD_TOL = 1e-30, 1e-60
DD_ORTH, QD_ORTH = 1e-28, 1e-58


@pytest.fixture(scope="module")
def zk():
    import torch
    import paper_2402_11868_amd as Z
    Z.load()
    ctx = Z.Context(0)
    yield Z, ctx, torch
    torch.cuda.synchronize()
    ctx.close()


def _dev(torch, planes):
    return [torch.from_numpy(np.ascontiguousarray(p)).to("cuda") for p in planes]


# ---------------------------------------------------------------- stage 1 --
@pytest.mark.parametrize("n", [1, 2, 3, 16, 33, 64, 100, 130])
def test_stage1_binary64(zk, n):
    Z, ctx, torch = zk
    log(f"stage1 n={n}")
    A = W.random_elements(n, 100 + n)
    (w, V), = Z.heev_fp64(ctx, [_dev(torch, [A])[0]])
    w = w.cpu().numpy()
    V = V.cpu().numpy()
    ref = np.linalg.eigvalsh(A)
    nrm = max(np.abs(ref).max(), 1e-300)
    u = 2.0 ** -53
    assert np.abs(w - ref).max() <= 16 * n * u * nrm
    assert np.abs(A @ V - V * w).max() <= 64 * n * u * nrm
    assert np.abs(V.conj().T @ V - np.eye(n)).max() <= 1e-8


def test_stage1_batch_of_equal_order(zk):
    Z, ctx, torch = zk
    mats = [W.random_elements(40, 200 + i) for i in range(5)]
    res = Z.heev_fp64(ctx, [_dev(torch, [A])[0] for A in mats])
    for A, (w, V) in zip(mats, res):
        assert np.abs(w.cpu().numpy() - np.linalg.eigvalsh(A)).max() <= 1e-12 * np.abs(A).sum()


def test_stage1_mixed_orders_one_call(zk):
    """Matrices of many orders in one call (orders around the 64-row chunk
    and 32-column panel edges; batches of different orders run concurrently
    on several streams), each checked against LAPACK."""
    Z, ctx, torch = zk
    orders = [2, 5, 31, 33, 64, 65, 97, 130, 200, 257]
    mats = [W.random_elements(n, 300 + n) for n in orders]
    res = Z.heev_fp64(ctx, [_dev(torch, [A])[0] for A in mats])
    u = 2.0 ** -53
    for n, A, (w, V) in zip(orders, mats, res):
        w, V = w.cpu().numpy(), V.cpu().numpy()
        ref = np.linalg.eigvalsh(A)
        nrm = np.abs(ref).max()
        log(f"mixed orders: n={n} |w - lapack| {np.abs(w - ref).max() / nrm:.2e}")
        assert np.abs(w - ref).max() <= 16 * n * u * nrm
        assert np.abs(A @ V - V * w).max() <= 64 * n * u * nrm
        assert np.abs(V.conj().T @ V - np.eye(n)).max() <= 1e-8


# ---------------------------------------------------------- dd, oracle ---
def test_c1_dd_against_golden(zk):
    """64x64 workload (designed spectrum, one eigenvalue 2^-20): all pairs vs stored oracle values."""
    Z, ctx, torch = zk
    import golden_io as G
    wl = W.workload(1)
    hdr, gold = G.load("c1")
    assert hdr["sha256"] == G.sha(wl["A"])
    log("c1 dd")
    res, = Z.heev(ctx, [_dev(torch, [wl["A"]])], limbs_out=2)
    out = gate([wl["A"]], res, gold, DD_TOL, orth_tol=DD_ORTH)
    log(f"c1: {out} iters={np.bincount(res.iters)}")


@pytest.mark.parametrize("n", [2, 3, 4, 17, 33, 56, 75, 96])
def test_dd_householder_family(zk, n):
    Z, ctx, torch = zk
    A = W.householder_hermitian(W.spectrum_c4(n), seed=W.seed_for(4, n))
    log(f"dd householder n={n}")
    ref = oracle.heev([A], want_vectors=False)
    res, = Z.heev(ctx, [_dev(torch, [A])], limbs_out=2)
    gate([A], res, ref.w_limbs, DD_TOL, orth_tol=DD_ORTH)


def test_dd_n1(zk):
    Z, ctx, torch = zk
    A = np.array([[0.3 + 0.7j]])
    res, = Z.heev(ctx, [_dev(torch, [A])], limbs_out=2)
    w, V = to_np(res)
    assert w[0, 0] == 0.3 and w[1, 0] == 0.0   # imaginary part of the diagonal ignored
    assert abs(abs(V[0, 0, 0]) - 1.0) == 0.0


@pytest.mark.parametrize("k,omega", [(39, 1), (59, 1j), (80, -1j), (100, -1)])
def test_dd_schmidt_pair(zk, k, omega):
    """The paper's Schmidt pair (Sec. 1, footnote 1): eigenvalues 1-eps and eps, eps = 2^-k, limb input."""
    Z, ctx, torch = zk
    planes, (eps, one_minus) = W.schmidt_pair(k, omega, limbs=2)
    res, = Z.heev(ctx, [_dev(torch, planes)], limbs_out=2)
    w, V = to_np(res)
    got = [Fraction(float(w[0, i])) + Fraction(float(w[1, i])) for i in range(2)]
    assert abs(got[0] - eps) <= Fraction(1, 10 ** 30)
    assert abs(got[1] - one_minus) <= Fraction(1, 10 ** 30)
    r, _ = oracle.residuals(planes, w, V)
    assert r.max() <= DD_TOL


def test_dd_schmidt_pair_binary64_alone_is_not_enough(zk):
    """Negative control: the binary64 stage alone cannot represent 1 - 2^-59."""
    Z, ctx, torch = zk
    planes, (eps, one_minus) = W.schmidt_pair(59, 1, limbs=2)
    (w, V), = Z.heev_fp64(ctx, [_dev(torch, planes)])
    w = w.cpu().numpy()
    assert abs(Fraction(float(w[0])) - eps) > Fraction(1, 10 ** 30) or abs(Fraction(float(w[1])) - one_minus) > Fraction(1, 10 ** 30)


@pytest.mark.parametrize("n,limbs,span", [(16, 1, 20), (64, 2, 60), (128, 1, 30)])
def test_dd_hadamard_exact(zk, n, limbs, span):
    """Exact spectrum with exact degeneracies and zero eigenvalues."""
    Z, ctx, torch = zk
    rng = np.random.Generator(np.random.PCG64(5000 + n))
    vals = []
    for _ in range(n - 6):
        vals.append(Fraction(int(rng.integers(1, 2 ** 12)), 2 ** (12 + int(rng.integers(0, span)))))
    vals += vals[:4] + [Fraction(0)] * 2
    h = W.hadamard_exact(vals, seed=n, limbs=limbs)
    log(f"hadamard n={n} L={limbs}")
    res, = Z.heev(ctx, [_dev(torch, h.planes)], limbs_out=2)
    ref = np.zeros((4, n))
    for k, x in enumerate(h.lam):
        f = float(x)
        ref[0, k] = f
        ref[1, k] = float(x - Fraction(f))
    gate(h.planes, res, ref, DD_TOL, orth_tol=DD_ORTH)


def test_dd_batch_mixed_sizes(zk):
    Z, ctx, torch = zk
    mats = [W.householder_hermitian(W.spectrum_c4(n), seed=W.seed_for(4, n) + 7) for n in (16, 48, 16, 32)]
    res = Z.heev(ctx, [_dev(torch, [A]) for A in mats], limbs_out=2)
    for A, r in zip(mats, res):
        gate([A], r, oracle.heev([A], want_vectors=False).w_limbs, DD_TOL, orth_tol=DD_ORTH)


def test_rqi_refine_from_lapack_pairs(zk):
    """Stage 2 alone, seeded with LAPACK binary64 pairs (test input, not a product path)."""
    Z, ctx, torch = zk
    n = 48
    A = W.householder_hermitian(W.spectrum_c4(n), seed=99)
    w0, V0 = np.linalg.eigh(A)
    res = Z.rqi_refine(ctx, _dev(torch, [A]), torch.from_numpy(w0).cuda(), torch.from_numpy(V0).cuda(), limbs_out=2)
    gate([A], res, oracle.heev([A], want_vectors=False).w_limbs, DD_TOL, orth_tol=DD_ORTH)


# ---------------------------------------------------------------- qd -----
@pytest.mark.parametrize("k", [59, 100])
def test_qd_schmidt_pair(zk, k):
    Z, ctx, torch = zk
    planes, (eps, one_minus) = W.schmidt_pair(k, 1j, limbs=2)
    res, = Z.heev(ctx, [_dev(torch, planes)], limbs_out=4)
    w, V = to_np(res)
    got = [sum((Fraction(float(w[l, i])) for l in range(4)), Fraction(0)) for i in range(2)]
    assert abs(got[0] - eps) <= Fraction(1, 10 ** 60)
    assert abs(got[1] - one_minus) <= Fraction(1, 10 ** 60)
    r, _ = oracle.residuals(planes, w, V)
    assert r.max() <= QD_TOL


@pytest.mark.parametrize("n,limbs,span", [(16, 4, 150), (32, 4, 120)])
def test_qd_hadamard_exact(zk, n, limbs, span):
    Z, ctx, torch = zk
    rng = np.random.Generator(np.random.PCG64(7000 + n))
    vals = [Fraction(int(rng.integers(1, 2 ** 40)), 2 ** (40 + int(rng.integers(0, span)))) for _ in range(n - 2)]
    vals += [Fraction(1) - Fraction(1, 2 ** 59), Fraction(1, 2 ** 59)]
    h = W.hadamard_exact(vals, seed=n + 1, limbs=limbs)
    res, = Z.heev(ctx, [_dev(torch, h.planes)], limbs_out=4)
    ref = np.zeros((4, n))
    for k, x in enumerate(h.lam):
        r = x
        for l in range(4):
            f = float(r)
            ref[l, k] = f
            r -= Fraction(f)
    gate(h.planes, res, ref, QD_TOL, orth_tol=QD_ORTH)


def test_qd_householder_n24(zk):
    Z, ctx, torch = zk
    A = W.householder_hermitian(W.spectrum_c4(24), seed=31)
    res, = Z.heev(ctx, [_dev(torch, [A])], limbs_out=4)
    gate([A], res, oracle.heev([A], want_vectors=False).w_limbs, QD_TOL, orth_tol=QD_ORTH)


# ------------------------------------------------------ FP32-MFMA start ----
def test_fp32_mfma_start_variant(zk):
    """Binary64 stage on the complex64-rounded input with FP32-MFMA GEMMs; the
    refinement reaches the same gates from the coarser start."""
    Z, ctx, torch = zk
    import golden_io as G
    wl = W.workload(1)
    hdr, gold = G.load("c1")
    d = _dev(torch, [wl["A"]])
    r64, = Z.heev(ctx, [d], limbs_out=2)
    r32, = Z.heev(ctx, [d], limbs_out=2, opts=Z.make_opts(init_fp32=1))
    out = gate([wl["A"]], r32, gold, DD_TOL, orth_tol=DD_ORTH)
    log(f"fp32 start: {out}; iterations fp64 start {np.bincount(r64.iters)}, fp32 start {np.bincount(r32.iters)}")
    assert np.mean(r32.iters) >= np.mean(r64.iters)
    A = W.householder_hermitian(W.spectrum_c4(130), seed=77)
    r, = Z.heev(ctx, [_dev(torch, [A])], limbs_out=2, opts=Z.make_opts(init_fp32=1))
    gate([A], r, oracle.heev([A], want_vectors=False).w_limbs, DD_TOL, orth_tol=DD_ORTH)


# ------------------------------------------------------------- errors ----
def test_errors_nan_and_bad_args(zk):
    Z, ctx, torch = zk
    import ctypes
    A = W.random_elements(8, 1)
    A[5, 2] = np.nan
    with pytest.raises(RuntimeError, match="EINVAL"):
        Z.heev(ctx, [_dev(torch, [A])], limbs_out=2)
    keep = []
    B = torch.from_numpy(W.random_elements(8, 2)).cuda()
    h = Z.herm(B, keep)
    h.lda = 4
    o, *_ = Z._alloc_out(8, 2, True, B.device, keep)
    rc = Z.load().zk_heev_dd(ctx.handle, 1, ctypes.byref(h), ctypes.byref(o), None)
    assert rc == Z.ZK_EINVAL
    h.lda = 8
    h.limbs = 3
    assert Z.load().zk_heev_dd(ctx.handle, 1, ctypes.byref(h), ctypes.byref(o), None) == Z.ZK_EINVAL


def test_enoconv_with_zero_iterations(zk):
    """max_iter = -1 (no shifted solve allowed): binary64 pairs miss 1e-30, status ZK_ENOCONV with flags."""
    Z, ctx, torch = zk
    A = W.householder_hermitian(W.spectrum_c4(20), seed=3)
    res, = Z.heev(ctx, [_dev(torch, [A])], limbs_out=2, opts=Z.make_opts(max_iter=-1))
    assert res.status == Z.ZK_ENOCONV
    assert all(i["iters"] == 0 and not (i["flags"] & Z.PAIR_CONVERGED) for i in res.info)
