"""The named workloads at their real shapes, through the C-ABI.

* clustered 1024: one 1024x1024 matrix with eigenvalues in clusters of 8
  (relative separation 1e-12, centres 1 .. 2^-50), in the launch
  configuration the benchmark times: all 1024 eigenvalues against stored
  oracle values, MPFR residuals of all 1024 pairs, the MPFR Gram matrix of all
  1024 vectors, and every pair's device-reported residual (the one the
  benchmark counts passing pairs by) against its MPFR residual.
* batch: 256 independent 128x128 matrices (geometric spectra 10^(-k/8) down to
  1e-16 with four exact 2-fold degeneracies each) in ONE zk_heev_dd call;
  every pair's device residual is gated; 16 members spread over the batch are
  gated in full against stored oracle eigenvalues, MPFR residuals and
  orthogonality of every pair, and device-vs-MPFR residual agreement.
* quad-double companions: 16 concurrent 256x256 requests through a session
  (4-limb Hadamard-family inputs carrying the quad-double spectrum {1-2^-59,
  2^-59} U 2^(-120k/254), exact in four binary64 limbs, so the true
  eigenvalues are known exactly), plus the binary64-input companion against
  stored oracle values.
* quad-double 2048: the 4-limb 2048x2048 input; the binary64 stage on the
  whole matrix and quad-double refinement of the 16 largest pairs
  (zk_rqi_refine), gated against the exact eigenvalues and eigenvectors.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W

from gpu_helpers import gate, log

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


def _exact_ref_limbs(lam):
    """(4, n) binary64 limbs of exact eigenvalues (ascending Fractions)."""
    ref = np.zeros((4, len(lam)))
    for k, x in enumerate(lam):
        r = x
        for l in range(4):
            f = float(r)
            ref[l, k] = f
            r -= Fraction(f)
    return ref


def _angle_sq_to_exact(V_limbs, k, e):
    """sin^2 of the angle between returned vector k (limb sum, exact) and the exact vector e (entries +-1, +-i)."""
    n = e.shape[0]
    pr = Fraction(0)
    pi = Fraction(0)
    nv = Fraction(0)
    er = np.real(e).astype(np.int64)
    ei = np.imag(e).astype(np.int64)
    xr = [Fraction(0)] * n
    xi = [Fraction(0)] * n
    for l in range(V_limbs.shape[0]):
        col = V_limbs[l, :, k]
        for i in range(n):
            xr[i] += Fraction(float(col[i].real))
            xi[i] += Fraction(float(col[i].imag))
    for i in range(n):
        # conj(e_i) x_i with e_i in {1, i, -1, -i}
        a, b = int(er[i]), int(ei[i])
        pr += a * xr[i] + b * xi[i]
        pi += a * xi[i] - b * xr[i]
        nv += xr[i] * xr[i] + xi[i] * xi[i]
    return 1 - (pr * pr + pi * pi) / (n * nv)


# ---------------------------------------------------------- clustered 1024 --
def test_clustered_1024_against_golden(zk):
    Z, ctx, torch = zk
    import golden_io as G
    A = W.workload(3)["A"]
    hdr, gold = G.load("c3")
    assert hdr["sha256"] == G.sha(A)
    log("clustered 1024 dd")
    stats = {}
    res, = Z.heev(ctx, [[torch.from_numpy(A).cuda()]], limbs_out=2, stats=stats)
    torch.cuda.synchronize()
    log(f"clustered 1024: iterations {stats['iters_hist'][:10]}, status {res.status}")
    rs = np.array([x["resid"] for x in res.info])
    log(f"clustered 1024: device residual > tol for {(rs > DD_TOL).sum()} pairs, max {rs.max():.3e}")
    # every eigenvalue, every vector: MPFR residuals, the whole Gram matrix and
    # the device residual of each pair against its MPFR value
    out = gate([A], res, gold, DD_TOL, orth_tol=DD_ORTH, dev_resid="agree")
    assert out["checked"] == 1024
    log(f"clustered 1024: {out}")


# ------------------------------------------------------------------ batch --
def test_batch_256_of_128(zk):
    Z, ctx, torch = zk
    import golden_io as G
    mats = [W.workload(2, index=i)["A"] for i in range(256)]
    dev = [torch.from_numpy(A).cuda() for A in mats]
    log("batch 256 x 128^2 dd")
    stats = {}
    res = Z.heev(ctx, [[d] for d in dev], limbs_out=2, stats=stats)
    torch.cuda.synchronize()
    log(f"batch: iterations {stats['iters_hist'][:8]}, rounds {stats['rounds']}")
    worst = 0.0
    for i, r in enumerate(res):
        hn = float(np.abs(r.w[0].cpu().numpy()).max())
        rs = max(x["resid"] for x in r.info)
        worst = max(worst, rs)
        assert r.status == Z.ZK_OK, f"matrix {i}: status {r.status}"
        assert rs <= DD_TOL, f"matrix {i}: device residual {rs:.3e}"
        assert hn > 0.0
    log(f"batch: max device residual {worst:.3e}")
    members = list(range(0, 256, 17))
    assert len(members) == 16 and all(G.exists(f"c2:{i}") for i in members), "stored batch oracle values missing"
    for i in members:
        hdr, gold = G.load(f"c2:{i}")
        assert hdr["sha256"] == G.sha(mats[i])
        out = gate([mats[i]], res[i], gold, DD_TOL, orth_tol=DD_ORTH, dev_resid="agree")
        log(f"batch member {i}: {out}")


# ------------------------------------------------- quad-double companions --
def _c5_companion(i, n=256):
    return W.hadamard_exact(W.spectrum_c5_dyadic(n), seed=W.seed_for(5, 100 + i), limbs=4)


def test_qd_companions_session(zk):
    Z, ctx, torch = zk
    comps = [_c5_companion(i) for i in range(16)]
    dev = [[torch.from_numpy(np.ascontiguousarray(p)).cuda() for p in h.planes] for h in comps]
    log("qd companions: 16 x 256^2 through the session")
    sess = Z.Session(ctx)
    tickets = [sess.submit(d, limbs_out=4) for d in dev]
    mixed = [sess.result(t) for t in tickets]
    lat = [sess.times(t) for t in tickets]
    log(f"qd companions: latencies (submit->done) {[round(c - a, 3) for a, b, c in lat]}")
    for i, (h, r) in enumerate(zip(comps, mixed)):
        bad = [(k, float(h.lam[k]), x["resid"], x["iters"], x["flags"]) for k, x in enumerate(r.info) if not (x["flags"] & 1)]
        assert r.status == Z.ZK_OK, f"request {i}: status {r.status}, unconverged (k, lam, resid, iters, flags) {bad[:8]}"
        ref = _exact_ref_limbs(h.lam)
        out = gate(h.planes, r, ref, QD_TOL, orth_tol=QD_ORTH)
        log(f"companion {i}: {out}")
    sess.close()
    # the first request alone gives the same bits
    alone, = Z.heev(ctx, [dev[0]], limbs_out=4)
    torch.cuda.synchronize()
    assert torch.equal(alone.w, mixed[0].w) and torch.equal(alone.V, mixed[0].V)


def test_qd_companion_binary64_input(zk):
    Z, ctx, torch = zk
    import golden_io as G
    if not G.exists("c5:256:0"):
        pytest.skip("stored oracle values for the binary64-input companion are missing")
    wl = W.workload(5, index=0, n=256)
    hdr, gold = G.load("c5:256:0")
    assert hdr["sha256"] == G.sha(wl["A"])
    log("qd companion, binary64 input")
    res, = Z.heev(ctx, [[torch.from_numpy(wl["A"]).cuda()]], limbs_out=4)
    out = gate([wl["A"]], res, gold, QD_TOL, orth_tol=QD_ORTH)
    log(f"companion L=1: {out} iters={np.bincount(res.iters)}")


# ----------------------------------------------------------- quad-double 2048 --
def test_qd_2048_refine_largest(zk):
    Z, ctx, torch = zk
    n, k = 2048, 16
    h = W.hadamard_exact(W.spectrum_c5_dyadic(n), seed=W.seed_for(5, 0), limbs=4)
    planes = [torch.from_numpy(np.ascontiguousarray(p)).cuda() for p in h.planes]
    log("qd 2048: binary64 stage")
    (w0, V0), = Z.heev_fp64(ctx, [planes])
    torch.cuda.synchronize()
    sel = torch.arange(n - k, n, device=w0.device)
    log("qd 2048: refinement of the 16 largest pairs")
    res = Z.rqi_refine(ctx, planes, w0[sel].contiguous(), V0[:, sel].contiguous(), limbs_out=4)
    torch.cuda.synchronize()
    assert res.status == Z.ZK_OK, [x for x in res.info if not (x["flags"] & 1)][:3]
    ref = _exact_ref_limbs(h.lam[n - k:])
    w = res.w.cpu().numpy()
    hn = float(h.lam[-1])
    for j in range(k):
        got = sum((Fraction(float(w[l, j])) for l in range(4)), Fraction(0))
        err = abs(got - h.lam[n - k + j])
        assert err <= Fraction(QD_TOL) * Fraction(hn), f"pair {j}: eigenvalue error {float(err):.3e}"
    V = res.V.cpu().numpy()
    E = h.vectors_unnormalised()[:, n - k:]
    for j in range(k):
        s2 = _angle_sq_to_exact(V, j, E[:, j])
        assert s2 <= Fraction(1, 10 ** 116), f"pair {j}: sin^2(angle) {float(s2):.3e}"
    r, _ = oracle.residuals(h.planes, w[:, :4], V[:, :, :4])
    assert r.max() <= QD_TOL * hn
    log(f"qd 2048: max residual (4 sampled) {r.max() / hn:.3e}, iterations {res.iters}")
