"""End-to-end stream of the bond matrices of the paper's introductory circuit
(Sec. 1, footnote 1): the 15 cuts of the 16-qubit state C^15-Z |+>^15 |->,
orders 2 .. 256, submitted together to one session (continuous batching),
under both refinements.  Every matrix has rank <= 2, so all but two of its
eigenvalues are exact zeros; the other two have the closed form
(1 +- sqrt(2F - 1)) / 2 (F = ||rho||_F^2, exact), pinned against the oracle in
test_workloads_circuit.py; across the last cut they are 1 - 2^-15 and 2^-15.
Bar: eigenvalues within 1e-30, MPFR residuals within 1e-30 and
orthonormality within 1e-28 on every pair of every cut."""
from decimal import Decimal
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W

from gpu_helpers import limb_sum_fraction, log
from test_workloads_circuit import closed_form_pair

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


@pytest.mark.parametrize("refine", [0, 1])
def test_circuit_bond_stream(zk, refine):
    Z, ctx, torch = zk
    n = 16
    mats = W.circuit_bond_matrices(n, seed=11)
    log(f"circuit stream n={n} refine={refine}: orders {[m['rho'].shape[0] for m in mats]}")
    sess = Z.Session(ctx, budget=1 << 30)
    opts = Z.make_opts(refine=refine)
    tickets = [sess.submit([torch.from_numpy(m["rho"]).cuda()], limbs_out=2, opts=opts) for m in mats]
    res = [sess.result(t) for t in tickets]
    sess.close()
    worst = 0.0
    for m, r in zip(mats, res):
        d = m["rho"].shape[0]
        assert r.status == Z.ZK_OK, f"cut {m['k']}: status {r.status}"
        w = r.w.cpu().numpy()
        V = r.V.cpu().numpy()
        lam = [limb_sum_fraction(w[:, j]) for j in range(d)]
        lo, hi = closed_form_pair(m["R"], n)
        dec = lambda x: Decimal(x.numerator) / Decimal(x.denominator)
        assert abs(dec(lam[-1]) - hi) <= Decimal(TOL), f"cut {m['k']}: top eigenvalue"
        assert abs(dec(lam[-2]) - lo) <= Decimal(TOL), f"cut {m['k']}: second eigenvalue"
        for x in lam[:-2]:
            assert abs(x) <= Fraction(TOL), f"cut {m['k']}: zero eigenvalue off by {float(x):.3e}"
        rs, _ = oracle.residuals([m["rho"]], w, V)
        assert rs.max() <= TOL, f"cut {m['k']}: residual {rs.max():.3e}"
        mo, md = oracle.gram(V)
        assert mo <= ORTH and md <= ORTH, f"cut {m['k']}: orthogonality {mo:.3e} / {md:.3e}"
        worst = max(worst, rs.max())
    eps = Fraction(1, 2 ** (n - 1))
    last = res[-1].w.cpu().numpy()
    got = sorted(limb_sum_fraction(last[:, j]) for j in range(2))
    assert abs(got[0] - eps) <= Fraction(TOL) and abs(got[1] - (1 - eps)) <= Fraction(TOL)
    log(f"circuit stream n={n} refine={refine}: {len(mats)} bond matrices, resid {worst:.2e}, "
        f"iterations {sorted(set(x['iters'] for r in res for x in r.info))}")
