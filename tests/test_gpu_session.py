"""Serving session: continuous batching, admission by footprint, alone-vs-mix invariance.

A request's result must be the same when it runs alone (one-shot zk_heev_dd)
and inside a mixed stream of requests of other sizes arriving while others are
on the GPU; the kernels work per pair, per cluster or per matrix, so the test
demands bitwise equality (stronger than the 1e-30 tolerance), and also checks
the tolerance against the oracle for a sample.
"""
import time

import numpy as np
import pytest

import oracle
import workloads as W

from gpu_helpers import gate, log

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


def _pool():
    mats = []
    for i, n in enumerate([16, 48, 32, 80, 16, 64, 24, 96]):
        mats.append(W.householder_hermitian(W.spectrum_c4(n), seed=W.seed_for(4, n) + 11 * i))
    return mats


def test_session_alone_vs_mix_bitwise(zk):
    Z, ctx, torch = zk
    mats = _pool()
    dev = [torch.from_numpy(A).cuda() for A in mats]
    alone = [Z.heev(ctx, [[d]], limbs_out=2)[0] for d in dev]
    torch.cuda.synchronize()
    sess = Z.Session(ctx, budget=64 << 20)
    tickets = []
    # staggered arrivals: half at once, the rest while the first ones iterate
    for d in dev[:4]:
        tickets.append(sess.submit([d]))
    time.sleep(0.05)
    for d in dev[4:]:
        tickets.append(sess.submit([d]))
        time.sleep(0.01)
    mixed = [sess.result(t) for t in tickets]
    for i, (a, m) in enumerate(zip(alone, mixed)):
        assert a.status == m.status
        assert torch.equal(a.w, m.w), f"request {i}: eigenvalues differ alone vs mix"
        assert torch.equal(a.V, m.V), f"request {i}: eigenvectors differ alone vs mix"
        assert [x["iters"] for x in a.info] == [x["iters"] for x in m.info]
    ts = [sess.times(t) for t in tickets]
    assert all(s <= ad <= d for (s, ad, d) in ts)
    log(f"latencies ms: {[round(1e3 * (d - s), 1) for (s, ad, d) in ts]}")
    # tolerance against the oracle for one member of the mix
    gate([mats[3]], mixed[3], oracle.heev([mats[3]], want_vectors=False).w_limbs, 1e-30, orth_tol=1e-28)
    sess.close()


def test_session_admission_and_errors(zk):
    Z, ctx, torch = zk
    import ctypes
    A = torch.from_numpy(W.householder_hermitian(W.spectrum_c4(64), seed=5)).cuda()
    # a budget below one request's footprint: refused at submit
    small = Z.Session(ctx, budget=1 << 16)
    with pytest.raises(RuntimeError, match="ENOMEM"):
        small.submit([A])
    small.close()
    # a budget that admits only one request at a time: all still complete, in order
    one = Z.Session(ctx, budget=2 * 64 * 64 * 16 * 4)
    ts = [one.submit([A]) for _ in range(3)]
    res = [one.result(t) for t in ts]
    times = [one.times(t) for t in ts]
    assert all(r.status in (Z.ZK_OK, Z.ZK_ENOCONV) for r in res)
    for (s0, a0, d0), (s1, a1, d1) in zip(times, times[1:]):
        assert a1 >= d0 - 1e-3, "second request admitted before the first finished under a one-request budget"
    for r in res[1:]:
        assert torch.equal(r.w, res[0].w)
    # unknown ticket
    rc, _ = one.poll(123456, 0)
    assert rc == Z.ZK_EINVAL
    one.close()


def test_session_qd_and_dd_mixed(zk):
    Z, ctx, torch = zk
    planes, (eps, one_minus) = W.schmidt_pair(100, 1j, limbs=2)
    dp = [torch.from_numpy(p).cuda() for p in planes]
    A = torch.from_numpy(W.householder_hermitian(W.spectrum_c4(24), seed=8)).cuda()
    sess = Z.Session(ctx)
    t1 = sess.submit(dp, limbs_out=4)
    t2 = sess.submit([A], limbs_out=2)
    r1, r2 = sess.result(t1), sess.result(t2)
    alone = Z.heev(ctx, [dp], limbs_out=4)[0]
    assert torch.equal(r1.w, alone.w)
    assert r2.status == Z.ZK_OK
    sess.close()
