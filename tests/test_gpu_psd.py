"""Rank-deficient positive semidefinite bond matrices rho = theta theta^H, the
input class of the MPS simulation the method serves (Sec. 1: a bond matrix of
an MPS is a reduced density matrix; its Schmidt coefficients are the square
roots of the eigenvalues, many of them zero or tiny).

Both refinements.  Checked by what holds at any size, since the oracle's
Jacobi at order 256 takes minutes:
* theta with small Gaussian-integer entries makes rho exact in binary64 with
  exactly m - r zero eigenvalues: those must come out below 1e-30 ||rho||_2;
* the trace and the squared Frobenius norm of rho (exact rationals of its
  binary64 entries) equal sum(lam) and sum(lam^2): with every eigenvalue
  within 1e-30 ||rho||_2 the sums agree to m 1e-30 ||rho||_2 and
  2 m 1e-30 ||rho||_2^2 (a collective double-double pin of the spectrum);
* agreement with LAPACK to binary64 accuracy; for the exact rho, no
  eigenvalue below -1e-30 ||rho||_2;
* MPFR residuals of every pair, each pair's device-reported residual against
  its MPFR value, and the MPFR Gram matrix of all vectors.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle

from gpu_helpers import check_device_residuals, limb_sum_fraction, log

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


def _rho(m, r, span, seed):
    rng = np.random.default_rng(seed)
    if span == 0:
        th = rng.integers(-8, 9, (m, r)) + 1j * rng.integers(-8, 9, (m, r))
    else:
        th = (rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))) * \
            (2.0 ** (-span * np.arange(r) / (r - 1)))[None, :]
    rho = th @ th.conj().T
    return (rho + rho.conj().T) / 2


def _exact_trace_frob(rho):
    tr = sum((Fraction(float(rho[i, i].real)) for i in range(rho.shape[0])), Fraction(0))
    re = rho.real.ravel()
    im = rho.imag.ravel()
    fr = sum((Fraction(float(x)) ** 2 for x in re), Fraction(0)) + sum((Fraction(float(x)) ** 2 for x in im), Fraction(0))
    return tr, fr


@pytest.mark.parametrize("refine", [0, 1])
@pytest.mark.parametrize("m,r,span", [(256, 128, 0), (256, 128, 40), (384, 96, 0)])
def test_psd_rank_deficient(zk, m, r, span, refine):
    """An exact null space of dimension m - r is one degenerate cluster: the
    per-pair iteration needs the offset shift after its first solve there."""
    Z, ctx, torch = zk
    rho = _rho(m, r, span, seed=1000 * m + r + span)
    log(f"psd m={m} r={r} span={span} refine={refine}")
    res, = Z.heev(ctx, [[torch.from_numpy(rho).cuda()]], limbs_out=2, opts=Z.make_opts(refine=refine))
    torch.cuda.synchronize()
    assert res.status == Z.ZK_OK
    w = res.w.cpu().numpy()
    V = res.V.cpu().numpy()
    lap = np.linalg.eigvalsh(rho)
    hn = float(np.max(np.abs(lap)))
    assert np.all(np.abs(w[0] - lap) <= 1e-13 * hn)
    lam = [limb_sum_fraction(w[:, k]) for k in range(m)]
    if span == 0:
        # exactly positive semidefinite (the graded rho is theta theta^H
        # rounded to binary64, whose tiny eigenvalues can be negative), with
        # exactly m - r zero eigenvalues (the lowest of the ascending order)
        assert min(lam) >= -Fraction(TOL) * Fraction(hn)
        zmax = max(abs(x) for x in lam[:m - r])
        assert zmax <= Fraction(TOL) * Fraction(hn), f"zero eigenvalue off by {float(zmax):.3e}"
    tr, fr = _exact_trace_frob(rho)
    dtr = abs(sum(lam, Fraction(0)) - tr)
    dfr = abs(sum((x * x for x in lam), Fraction(0)) - fr)
    assert dtr <= m * Fraction(TOL) * Fraction(hn), f"trace off by {float(dtr) / hn:.3e} ||rho||"
    assert dfr <= 2 * m * Fraction(TOL) * Fraction(hn) ** 2, f"Frobenius norm off by {float(dfr) / hn ** 2:.3e} ||rho||^2"
    # every pair: MPFR residual, device residual against it, whole Gram matrix
    rs, _ = oracle.residuals([rho], w, V)
    assert rs.max() <= TOL * hn, f"residual {rs.max() / hn:.3e} ||rho|| (k={int(rs.argmax())})"
    dd = check_device_residuals(res, np.arange(m), rs, hn, mode="agree" if refine == 0 else "bound")
    mo, md = oracle.gram(V)
    assert mo <= ORTH and md <= ORTH, f"orthogonality {mo:.3e} / {md:.3e}"
    log(f"psd m={m} r={r} span={span} refine={refine}: trace {float(dtr) / hn:.2e}, "
        f"frob {float(dfr) / hn ** 2:.2e}, resid {rs.max() / hn:.2e}, device-vs-MPFR {dd:.1e}, "
        f"orth {max(mo, md):.1e}")



def test_psd_exact_rank_deficient_qd(zk):
    """The same exact null space in quad-double (bar 1e-60 ||rho||_2): the
    exact zeros, the trace identity, MPFR residuals of every pair and
    orthonormality of all vectors."""
    Z, ctx, torch = zk
    m, r = 128, 48
    qtol, qorth = 1e-60, 1e-58
    rho = _rho(m, r, 0, seed=1000 * m + r)
    log(f"psd qd m={m} r={r}")
    res, = Z.heev(ctx, [[torch.from_numpy(rho).cuda()]], limbs_out=4)
    torch.cuda.synchronize()
    assert res.status == Z.ZK_OK
    w = res.w.cpu().numpy()
    V = res.V.cpu().numpy()
    hn = float(np.max(np.abs(np.linalg.eigvalsh(rho))))
    lam = [limb_sum_fraction(w[:, k]) for k in range(m)]
    assert max(abs(x) for x in lam[:m - r]) <= Fraction(qtol) * Fraction(hn)
    tr, _ = _exact_trace_frob(rho)
    assert abs(sum(lam, Fraction(0)) - tr) <= m * Fraction(qtol) * Fraction(hn)
    rs, _ = oracle.residuals([rho], w, V)
    assert rs.max() <= qtol * hn, f"residual {rs.max() / hn:.3e} ||rho||"
    check_device_residuals(res, np.arange(m), rs, hn, mode="agree", slack=1e-62)
    mo, md = oracle.gram(V)
    assert mo <= qorth and md <= qorth, f"orthogonality {mo:.3e} / {md:.3e}"
    log(f"psd qd m={m} r={r}: resid {rs.max() / hn:.2e}, iterations {sorted(set(x['iters'] for x in res.info))}")
