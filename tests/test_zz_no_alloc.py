"""zk_heev_dd_noalloc (workspace from the library's static scratch array, no
device allocation during the call) against zk_heev_dd on the same inputs.

Two calls in a row through the C-ABI, the second with a smaller input, each
compared with zk_heev_dd: eigenvalues to 1e-30 ||H||_2; eigenvectors, which
are not unique below residual / gap, checked for validity in MPFR (residual
and orthonormality at the same bar).  The context's own workspace must be untouched by the
no-allocation calls, and a call too large for the array is refused before
any work.
"""
import numpy as np
import pytest

import workloads as W

from gpu_helpers import gate, log

pytestmark = pytest.mark.gpu

TOL = 1e-30


@pytest.fixture(scope="module")
def zk():
    import torch
    import paper_2402_11868_amd as Z
    Z.load()
    ctx = Z.Context(0)
    yield Z, ctx, torch
    torch.cuda.synchronize()
    ctx.close()


def _mats(sizes, salt):
    return [W.householder_hermitian(W.spectrum_c4(n), seed=W.seed_for(4, n) + 977 * salt + i)
            for i, n in enumerate(sizes)]


def _compare(A, ref, got):
    """Eigenvalues are unique: the two results agree to 1e-30 ||H||_2.  The
    eigenvectors are fixed only up to phase and, for pairs whose gap is
    small, up to residual / gap (both results are valid dd decompositions, and
    the number of shifted factorisations running at once, which the smaller
    workspace limits, may change the order in which cluster members converge);
    so each vector must be a valid one: MPFR residual <= 1e-30 ||H||_2 and an
    orthonormal basis to 100 x 1e-30.  Returns whether the limbs are bitwise
    equal (logged, not required)."""
    wr = ref.w.cpu().numpy()
    hn = float(np.abs(wr[0]).max())
    out = gate([A], got, wr, TOL, orth_tol=100 * TOL)
    wg, Vg = got.w.cpu().numpy(), got.V.cpu().numpy()
    same = bool(np.array_equal(wr, wg) and np.array_equal(ref.V.cpu().numpy(), Vg))
    log(f"n={A.shape[0]}: |dw| {out['eig_err']:.2e}, resid {out['resid']:.2e}, orth {out['orth']:.2e} "
        f"(relative to ||H||_2 = {hn:.3e}), bitwise equal {same}")
    return same


@pytest.mark.parametrize("sizes", [[200, 96], [64]])
def test_noalloc_matches_heev_dd(zk, sizes):
    Z, ctx, torch = zk
    mats = _mats(sizes, len(sizes))
    dev = [torch.from_numpy(A).cuda() for A in mats]
    ref = Z.heev(ctx, [[d] for d in dev], limbs_out=2)
    torch.cuda.synchronize()
    held0 = ctx.memory()["held"]
    got = Z.heev(ctx, [[d] for d in dev], limbs_out=2, noalloc=True)
    torch.cuda.synchronize()
    assert ctx.memory()["held"] == held0, "the no-allocation call changed the context's workspace"
    for i, A in enumerate(mats):
        assert got[i].status == ref[i].status == Z.ZK_OK
        _compare(A, ref[i], got[i])


def test_noalloc_two_calls_in_a_row_shrinking(zk):
    Z, ctx, torch = zk
    big = [torch.from_numpy(A).cuda() for A in _mats([320], 7)]
    small = [torch.from_numpy(A).cuda() for A in _mats([48, 40], 8)]
    g1 = Z.heev(ctx, [[d] for d in big], limbs_out=2, noalloc=True)
    g2 = Z.heev(ctx, [[d] for d in small], limbs_out=2, noalloc=True)
    torch.cuda.synchronize()
    r1 = Z.heev(ctx, [[d] for d in big], limbs_out=2)
    r2 = Z.heev(ctx, [[d] for d in small], limbs_out=2)
    torch.cuda.synchronize()
    for ref, got, d in zip(r1 + r2, g1 + g2, big + small):
        assert got.status == Z.ZK_OK
        _compare(d.cpu().numpy(), ref, got)


def test_noalloc_refuses_what_does_not_fit(zk):
    Z, ctx, torch = zk
    A = torch.from_numpy(_mats([700], 9)[0]).cuda()
    held0 = ctx.memory()["held"]
    with pytest.raises(RuntimeError, match="ZK_ENOMEM"):
        Z.heev(ctx, [[A]], limbs_out=2, noalloc=True)
    assert "scratch" in ctx.last_error()
    assert ctx.memory()["held"] == held0
    # the context still works afterwards, on both entry points
    B = torch.from_numpy(_mats([32], 10)[0]).cuda()
    r = Z.heev(ctx, [[B]], limbs_out=2)
    g = Z.heev(ctx, [[B]], limbs_out=2, noalloc=True)
    torch.cuda.synchronize()
    _compare(B.cpu().numpy(), r[0], g[0])
