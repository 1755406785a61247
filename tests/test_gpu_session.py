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


def test_session_queue_full_and_cancel_on_destroy(zk):
    """A bounded queue refuses with ZK_EAGAIN when full; destroying the session
    cancels what is pending, and a thread blocked in zk_session_poll at that
    moment wakes with ZK_ECANCELED (the session stays alive until it has left)."""
    Z, ctx, torch = zk
    import threading
    mats = [torch.from_numpy(W.householder_hermitian(W.spectrum_c4(512), seed=21 + i)).cuda() for i in range(7)]
    # each order-512 request's footprint is about 25 MB: the budget admits one
    # at a time, the queue holds two more
    sess = Z.Session(ctx, budget=40 << 20, max_queue=2)
    sess.submit([mats[0]])
    time.sleep(0.01)
    refused = 0
    waiting = []
    for d in mats[1:]:
        try:
            waiting.append(sess.submit([d]))
        except RuntimeError as e:
            assert "EAGAIN" in str(e)
            refused += 1
    assert refused >= 1, "a queue bounded at 2 accepted 6 requests while one was running"
    got = {}
    entering = threading.Event()

    def poller():
        entering.set()
        got["rc"] = sess.poll(waiting[-1], -1)[0]

    th = threading.Thread(target=poller)
    th.start()
    assert entering.wait(10)
    time.sleep(0.05)   # the poller is blocked inside zk_session_poll (ctypes drops the GIL)
    sess.close()
    th.join(timeout=60)
    assert not th.is_alive(), "poller still blocked after destroy"
    assert got["rc"] == Z.ZK_ECANCELED, f"poller woke with {Z.status_str(got['rc'])}"
    log(f"queue-full refusals {refused}, poller woke with {Z.status_str(got['rc'])}")


def test_failed_call_gives_back_its_memory(zk):
    """A call that runs out of budget part-way (for instance after the
    iterate storage of its matrix was taken, before a shifted-LU slot or the
    Gram-Schmidt plan fits) must give that storage back: after the failed
    call the context holds no per-call memory, and a repeated failure does
    not grow what it holds."""
    Z, ctx, torch = zk
    n = 64
    A = torch.from_numpy(W.householder_hermitian(W.spectrum_c4(n), seed=31)).cuda()
    lib = Z.load()
    full = lib.zk_workspace_bytes(n, 2, 1) + (1 << 20)
    seen = 0
    for cut in range(0, 1600 << 10, 32 << 10):
        c = Z.Context(0, budget=full - cut)
        try:
            try:
                Z.heev(c, [[A]], limbs_out=2)
                assert c.memory()["transient"] == 0
                continue
            except RuntimeError as e:
                assert "ENOMEM" in str(e), str(e)
            m1 = c.memory()
            assert m1["transient"] == 0, f"budget {full - cut}: {m1['transient']} bytes kept after a failed call"
            with pytest.raises(RuntimeError, match="ENOMEM"):
                Z.heev(c, [[A]], limbs_out=2)
            m2 = c.memory()
            assert m2["held"] == m1["held"] and m2["transient"] == 0, f"budget {full - cut}: {m1} -> {m2}"
            seen += 1
        finally:
            c.close()
    assert seen >= 1
    log(f"failed-call budgets checked: {seen}")


def test_engines_share_lu_slots_under_tight_budget(zk):
    """Double-double, quad-double and all-pairs requests in one session whose
    context budget is tight, so the all-pairs engine gives back the shifted-LU
    slots that the two Rayleigh-quotient engines laid out for their own
    limbs: every result still equals the one computed alone."""
    Z, ctx, torch = zk
    mats = [W.householder_hermitian(W.spectrum_c4(n), seed=W.seed_for(4, n) + 41 * i)
            for i, n in enumerate([96, 64, 80, 96, 48, 64])]
    dev = [torch.from_numpy(A).cuda() for A in mats]
    kinds = [(2, 0), (4, 0), (2, 1), (2, 0), (4, 0), (2, 1)]
    big = Z.Context(0)
    alone = []
    for d, (L, rf) in zip(dev, kinds):
        alone.append(Z.heev(big, [[d]], limbs_out=L, opts=Z.make_opts(refine=rf))[0])
    torch.cuda.synchronize()
    big.close()
    tight = Z.Context(0, budget=24 << 20)
    sess = Z.Session(tight, budget=24 << 20)
    tickets = []
    for d, (L, rf) in zip(dev, kinds):
        tickets.append(sess.submit([d], limbs_out=L, opts=Z.make_opts(refine=rf)))
        time.sleep(0.003)
    mixed = [sess.result(t) for t in tickets]
    sess.close()
    for i, (a, m) in enumerate(zip(alone, mixed)):
        assert m.status == a.status, f"request {i}: status {m.status} vs {a.status}"
        assert torch.equal(a.w, m.w) and torch.equal(a.V, m.V), f"request {i}: result differs under the tight budget"
    log(f"tight budget: high water {tight.memory()['high_water']} of {24 << 20}")
    tight.close()
