"""Parity of the all-pairs refinement (zk_heev_dd_allpairs) with the MPFR oracle.

Same bar as the Rayleigh-quotient path: eigenvalue error and residual
||H v - lam v|| / ||v|| <= 1e-30 ||H||_2, orthogonality <= 1e-28, evaluated
exactly on the returned limbs.  The cases cover the designed 64x64 workload,
the clustered 1024x1024 workload (clusters of 8 at relative separation 1e-12
with centres down to 2^-50), the batch of 256 matrices of order 128, exact
degeneracies and zero eigenvalues, limb inputs, n = 1 and mixed orders.
"""
import time
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W

from gpu_helpers import gate, log, to_np

pytestmark = pytest.mark.gpu

DD_TOL, DD_ORTH = 1e-30, 1e-28


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
    return [torch.from_numpy(np.ascontiguousarray(p)).cuda() for p in planes]


def _iters(res):
    return sorted(set(int(x["iters"]) for x in res.info))


def test_allpairs_c1_against_golden(zk):
    Z, ctx, torch = zk
    import golden_io as G
    wl = W.workload(1)
    hdr, gold = G.load("c1")
    assert hdr["sha256"] == G.sha(wl["A"])
    log("all-pairs c1")
    res, = Z.heev_allpairs(ctx, [_dev(torch, [wl["A"]])])
    assert res.status == Z.ZK_OK
    out = gate([wl["A"]], res, gold, DD_TOL, orth_tol=DD_ORTH)
    log(f"all-pairs c1: {out} iterations {_iters(res)}")


@pytest.mark.parametrize("n", [2, 3, 17, 75])
def test_allpairs_householder_family(zk, n):
    Z, ctx, torch = zk
    A = W.householder_hermitian(W.spectrum_c4(n), seed=W.seed_for(4, n))
    log(f"all-pairs householder n={n}")
    res, = Z.heev_allpairs(ctx, [_dev(torch, [A])])
    assert res.status == Z.ZK_OK
    gate([A], res, oracle.heev([A], want_vectors=False).w_limbs, DD_TOL, orth_tol=DD_ORTH)


def test_allpairs_n1(zk):
    Z, ctx, torch = zk
    A = np.array([[0.3 + 0.7j]])
    res, = Z.heev_allpairs(ctx, [_dev(torch, [A])])
    w, V = to_np(res)
    assert w[0, 0] == 0.3 and w[1, 0] == 0.0
    assert abs(abs(V[0, 0, 0]) - 1.0) == 0.0


def test_allpairs_schmidt_pair(zk):
    """The paper's Schmidt pair (Sec. 1, footnote 1) with eps = 2^-59 in a two-limb input."""
    Z, ctx, torch = zk
    planes, (eps, one_minus) = W.schmidt_pair(59, 1j, limbs=2)
    res, = Z.heev_allpairs(ctx, [_dev(torch, planes)])
    w, V = to_np(res)
    got = [Fraction(float(w[0, i])) + Fraction(float(w[1, i])) for i in range(2)]
    assert abs(got[0] - eps) <= Fraction(1, 10 ** 30)
    assert abs(got[1] - one_minus) <= Fraction(1, 10 ** 30)
    r, _ = oracle.residuals(planes, w, V)
    assert r.max() <= DD_TOL


@pytest.mark.parametrize("n,limbs,span", [(16, 1, 20), (64, 2, 60), (128, 1, 30)])
def test_allpairs_hadamard_exact(zk, n, limbs, span):
    """Exact spectrum with exact degeneracies and zero eigenvalues."""
    Z, ctx, torch = zk
    rng = np.random.Generator(np.random.PCG64(5000 + n))
    vals = []
    for _ in range(n - 6):
        vals.append(Fraction(int(rng.integers(1, 2 ** 12)), 2 ** (12 + int(rng.integers(0, span)))))
    vals += vals[:4] + [Fraction(0)] * 2
    h = W.hadamard_exact(vals, seed=n, limbs=limbs)
    log(f"all-pairs hadamard n={n} L={limbs}")
    res, = Z.heev_allpairs(ctx, [_dev(torch, h.planes)])
    ref = np.zeros((4, n))
    for k, x in enumerate(h.lam):
        f = float(x)
        ref[0, k] = f
        ref[1, k] = float(x - Fraction(f))
    assert res.status == Z.ZK_OK
    out = gate(h.planes, res, ref, DD_TOL, orth_tol=DD_ORTH)
    log(f"all-pairs hadamard n={n}: {out} iterations {_iters(res)}")


def test_allpairs_mixed_orders(zk):
    Z, ctx, torch = zk
    mats = [W.householder_hermitian(W.spectrum_c4(n), seed=W.seed_for(4, n) + 7) for n in (16, 48, 16, 32)]
    res = Z.heev_allpairs(ctx, [_dev(torch, [A]) for A in mats])
    for A, r in zip(mats, res):
        assert r.status == Z.ZK_OK
        gate([A], r, oracle.heev([A], want_vectors=False).w_limbs, DD_TOL, orth_tol=DD_ORTH)


def test_allpairs_batch_256_of_128(zk):
    Z, ctx, torch = zk
    import golden_io as G
    mats = [W.workload(2, index=i)["A"] for i in range(256)]
    log("all-pairs batch 256 x 128^2")
    res = Z.heev_allpairs(ctx, [[torch.from_numpy(A).cuda()] for A in mats])
    torch.cuda.synchronize()
    worst = 0.0
    for i, r in enumerate(res):
        rs = max(x["resid"] for x in r.info)
        worst = max(worst, rs)
        assert r.status == Z.ZK_OK, f"matrix {i}: status {r.status}"
        assert rs <= DD_TOL, f"matrix {i}: device residual {rs:.3e}"
    log(f"all-pairs batch: max device residual {worst:.3e}, iterations {sorted(set(_iters(r)[0] for r in res))}")
    for i in range(0, 256, 17):
        hdr, gold = G.load(f"c2:{i}")
        assert hdr["sha256"] == G.sha(mats[i])
        out = gate([mats[i]], res[i], gold, DD_TOL, orth_tol=DD_ORTH, dev_resid="bound")
        log(f"all-pairs batch member {i}: {out}")


def test_allpairs_clustered_1024_against_golden(zk):
    Z, ctx, torch = zk
    import golden_io as G
    A = W.workload(3)["A"]
    hdr, gold = G.load("c3")
    assert hdr["sha256"] == G.sha(A)
    log("all-pairs clustered 1024")
    res, = Z.heev_allpairs(ctx, [[torch.from_numpy(A).cuda()]])
    torch.cuda.synchronize()
    rs = np.array([x["resid"] for x in res.info])
    log(f"all-pairs clustered 1024: status {res.status}, iterations {_iters(res)}, max device residual {rs.max():.3e}")
    assert res.status == Z.ZK_OK
    # every pair: MPFR residuals, the whole Gram matrix, device residual as an upper bound
    out = gate([A], res, gold, DD_TOL, orth_tol=DD_ORTH, dev_resid="bound")
    assert out["checked"] == 1024
    log(f"all-pairs clustered 1024: {out}")


def test_allpairs_refine_option_and_session(zk):
    """zk_heev_dd with opts.refine = 1 is the all-pairs entry point; session
    requests with refine = 1 run in the all-pairs engine with continuous
    batching (a request that arrives while others iterate joins at the next
    whole-basis iteration) and give the same bits as alone."""
    Z, ctx, torch = zk
    mats = [W.householder_hermitian(W.spectrum_c4(n), seed=W.seed_for(4, n) + 13 * i)
            for i, n in enumerate([16, 48, 32, 80, 16, 64, 24, 96])]
    dev = [torch.from_numpy(A).cuda() for A in mats]
    opts = Z.make_opts(refine=1)
    alone = [Z.heev_allpairs(ctx, [[d]])[0] for d in dev]
    via_opt, = Z.heev(ctx, [[dev[3]]], limbs_out=2, opts=opts)
    torch.cuda.synchronize()
    assert torch.equal(via_opt.w, alone[3].w) and torch.equal(via_opt.V, alone[3].V)
    sess = Z.Session(ctx, budget=256 << 20)
    tickets = []
    for d in dev[:4]:
        tickets.append(sess.submit([d], opts=opts))
    time.sleep(0.02)
    for d in dev[4:]:
        tickets.append(sess.submit([d], opts=opts))
        time.sleep(0.005)
    mixed = [sess.result(t) for t in tickets]
    sess.close()
    for i, (a, m) in enumerate(zip(alone, mixed)):
        assert m.status == Z.ZK_OK, f"request {i}: status {m.status}"
        assert torch.equal(a.w, m.w), f"request {i}: eigenvalues differ alone vs mix"
        assert torch.equal(a.V, m.V), f"request {i}: eigenvectors differ alone vs mix"
    for i in (0, 7):
        gate([mats[i]], mixed[i], oracle.heev([mats[i]], want_vectors=False).w_limbs, DD_TOL, orth_tol=DD_ORTH)
    with pytest.raises(RuntimeError):
        Z.heev(ctx, [[dev[0]]], limbs_out=4, opts=opts)


def test_dilation_shared_eigenvalues_both_refinements(zk):
    """K = [[0, T], [T^H, 0]] with T (2 x 4) of orthonormal dyadic rows: the
    eigenvalues are exactly -1, -1, 0, 0, 1, 1, and the tridiagonal of such
    dilations splits into blocks that share an eigenvalue.  The binary64
    stage must return independent vectors (it once returned one vector twice
    there), and both refinements must reach the exact spectrum."""
    Z, ctx, torch = zk
    T = 0.5 * np.array([[1, 1j, -1, 1j], [1, -1j, 1, 1j]])
    K = np.zeros((6, 6), dtype=np.complex128)
    K[:2, 2:] = T
    K[2:, :2] = T.conj().T
    Kd = torch.from_numpy(K).cuda()
    (w0, V0), = Z.heev_fp64(ctx, [[Kd]])
    V0 = V0.cpu().numpy()
    assert np.abs(V0.conj().T @ V0 - np.eye(6)).max() <= 1e-13
    ref = np.zeros((4, 6))
    ref[0] = [-1, -1, 0, 0, 1, 1]
    for opts in (Z.make_opts(refine=0), Z.make_opts(refine=1)):
        r, = Z.heev(ctx, [[Kd]], limbs_out=2, opts=opts)
        assert r.status == Z.ZK_OK
        gate([K], r, ref, DD_TOL, orth_tol=DD_ORTH)
