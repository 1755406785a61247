"""Shared helpers of the GPU tests: run the HIP path, check it against the oracle."""
from __future__ import annotations

import sys
from fractions import Fraction

import numpy as np

import oracle

# The device residual (exact products, cascaded double-double sums) must agree
# with the MPFR residual of the returned limbs to this fraction of ||H||_2: two
# orders below the 1e-30 gate, so a pair the device counts as passing passes.
DEV_RESID_AGREE = 1e-32


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def to_np(res):
    w = res.w.cpu().numpy()
    V = res.V.cpu().numpy() if res.V is not None else None
    return w, V


def limb_sum_fraction(limbs) -> Fraction:
    return sum((Fraction(float(x)) for x in limbs), Fraction(0))


def eig_errors(w_limbs: np.ndarray, ref_limbs: np.ndarray) -> np.ndarray:
    """|w_k - ref_k| for ascending eigenvalues, exact on the limb sums (as float)."""
    out = np.zeros(w_limbs.shape[1])
    for k in range(w_limbs.shape[1]):
        out[k] = float(abs(limb_sum_fraction(w_limbs[:, k]) - limb_sum_fraction(ref_limbs[:, k])))
    return out


def check_device_residuals(res, idx, r_mpfr, hn: float, mode: str = "agree",
                           slack: float = DEV_RESID_AGREE) -> float:
    """Per pair: the residual the device reports (info.resid, relative to ||H||_2)
    against the MPFR residual of the same returned limbs.
    mode "agree": |device - MPFR| <= slack ||H||_2;
    mode "bound": MPFR <= device + slack ||H||_2 (the device value may only
    overstate the residual, so a pair counted as passing by it passes).
    Returns the largest |device - MPFR| relative to ||H||_2."""
    dev = np.array([res.info[int(k)]["resid"] for k in idx]) * hn
    diff = np.abs(dev - r_mpfr)
    under = r_mpfr - dev
    bad = diff if mode == "agree" else under
    j = int(bad.argmax()) if len(bad) else 0
    assert bad.max(initial=0.0) <= slack * hn, (
        f"device residual ({mode}) fails against MPFR: pair {int(idx[j])} device {dev[j] / hn:.3e} "
        f"MPFR {r_mpfr[j] / hn:.3e} (relative to ||H||_2)")
    return float(diff.max(initial=0.0) / hn)


def gate(planes, res, ref_w_limbs, tol: float, check_vectors: bool = True, orth_tol: float | None = None,
         sample=None, dev_resid: str | None = None):
    """Gate a GPU result against the oracle.

    eigenvalues: |lam_hat - lam| <= tol ||H||_2 (normwise, ||H||_2 = max |lam|)
    residuals:   ||H v - lam_hat v|| / ||v|| <= tol ||H||_2, evaluated in MPFR on the returned limbs
    orthogonality (if orth_tol): max |v_i^H v_j|, | ||v_i||^2 - 1 | <= orth_tol
    dev_resid ("agree" / "bound"): every checked pair's device-reported residual
               against the MPFR one (check_device_residuals)
    """
    w, V = to_np(res)
    hn = float(np.max(np.abs(ref_w_limbs[0])))
    hn = hn if hn > 0 else 1.0
    err = eig_errors(w, ref_w_limbs)
    kw = int(err.argmax())
    assert err.max() <= tol * hn, (f"eigenvalue error {err.max():.3e} > {tol * hn:.3e} (k={kw}, "
                                   f"info={res.info[kw]}, iters={np.bincount(res.iters)})")
    out = {"eig_err": err.max() / hn}
    if check_vectors and V is not None:
        idx = np.arange(V.shape[2]) if sample is None else np.asarray(sample)
        r, vn = oracle.residuals(planes, w[:, idx], V[:, :, idx])
        assert np.all(np.isfinite(r))
        assert r.max() <= tol * hn, f"residual {r.max():.3e} > {tol * hn:.3e} (k={int(idx[r.argmax()])})"
        out["resid"] = r.max() / hn
        out["checked"] = len(idx)
        if dev_resid:
            out["dev_resid_diff"] = check_device_residuals(res, idx, r, hn, mode=dev_resid)
        if orth_tol is not None:
            mo, md = oracle.gram(V[:, :, idx])
            assert mo <= orth_tol and md <= orth_tol, f"orthogonality {mo:.3e}/{md:.3e} > {orth_tol:.1e}"
            out["orth"] = max(mo, md)
    return out
