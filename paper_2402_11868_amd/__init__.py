"""Python binding of libzk (the C-ABI declared in include/zk.h).

Argument marshalling only: every step of the eigendecomposition runs in the
HIP kernels of ``libzk.so``.  PyTorch supplies device memory and the HIP
stream.  There is no CPU fallback: importing this package without the built
library, or calling it without a GPU, raises.

Matrices are passed as torch complex128 CUDA tensors of shape (n, n) holding
the logical matrix A[i, j]; the binding hands the library a column-major copy
(only the lower triangle is read).  Limb inputs are lists of such tensors
whose exact sum is the matrix.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

import torch  # noqa: F401  -- loads torch's HIP runtime first; libzk binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libzk.so")

ZK_OK, ZK_ENOCONV, ZK_EINVAL, ZK_ENOMEM, ZK_EDEVICE, ZK_EAGAIN, ZK_ECANCELED, ZK_EINTERNAL = 0, 1, -1, -2, -3, -4, -5, -6
PAIR_CONVERGED, PAIR_REORTH, PAIR_PIVOT_GUARD, PAIR_NAN = 1, 2, 4, 8


class ZkHerm(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("lda", ctypes.c_int), ("limbs", ctypes.c_int),
                ("plane", ctypes.c_void_p * 4)]


class ZkPairInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("flags", ctypes.c_int32), ("cluster", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("resid", ctypes.c_double)]


class ZkEigOut(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("ldv", ctypes.c_int), ("limbs", ctypes.c_int),
                ("w", ctypes.c_void_p * 4), ("v", ctypes.c_void_p * 4), ("info", ctypes.POINTER(ZkPairInfo))]


class ZkEigOutMp(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("ldv", ctypes.c_int), ("limbs", ctypes.c_int),
                ("w", ctypes.c_void_p), ("v", ctypes.c_void_p), ("info", ctypes.POINTER(ZkPairInfo))]


class ZkMat(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("n", ctypes.c_int), ("lda", ctypes.c_int), ("limbs", ctypes.c_int),
                ("plane", ctypes.c_void_p * 4)]


class ZkSvdOut(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("n", ctypes.c_int), ("limbs", ctypes.c_int), ("s", ctypes.c_void_p * 4),
                ("u", ctypes.c_void_p * 4), ("ldu", ctypes.c_int), ("v", ctypes.c_void_p * 4), ("ldv", ctypes.c_int),
                ("info", ctypes.POINTER(ZkPairInfo))]


class ZkOpts(ctypes.Structure):
    _fields_ = [("init_fp32", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("cluster_tol", ctypes.c_double), ("want_vectors", ctypes.c_int), ("reorth", ctypes.c_int),
                ("refine", ctypes.c_int), ("shifted_solve", ctypes.c_int)]


KERNEL_CLASSES = ["lu_update", "lu_panel", "lu_trsm", "backsolve", "rq", "gs", "reorth", "stage1", "her2k", "hemv",
                  "build", "trd_vec", "tridiag", "backt", "ap_resid", "ap_fgemm", "ap_ddgemm", "ap_other"]

EXPORTED = ["zk_prof_enable", "zk_prof_classes", "zk_prof_reset", "zk_prof_read", "zk_opts_default", "zk_ctx_create", "zk_ctx_destroy", "zk_status_str", "zk_ctx_last_error",
            "zk_workspace_bytes", "zk_heev_dd", "zk_heev_qd", "zk_heev_dd_allpairs", "zk_svd_dd", "zk_mps_two_site_dd", "zk_heev_fp64", "zk_rqi_refine",
            "zk_session_create", "zk_session_submit", "zk_session_poll", "zk_session_times", "zk_session_destroy",
            "zk_ctx_memory", "zk_ctx_last_stats", "zk_heev_dd_noalloc", "zk_heev_mp",
            "zk_mps_create", "zk_mps_destroy", "zk_mps_apply1", "zk_mps_apply2", "zk_mps_bond", "zk_mps_site",
            "zk_mps_latencies"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libzk.so (raises OSError if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"libzk.so not built at {path}; run python -m paper_2402_11868_amd.build")
    lib = ctypes.CDLL(path)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.zk_opts_default.argtypes = [ctypes.POINTER(ZkOpts)]
    lib.zk_opts_default.restype = None
    lib.zk_ctx_create.argtypes = [I, P, ctypes.c_size_t, ctypes.POINTER(P)]
    lib.zk_ctx_destroy.argtypes = [P]
    lib.zk_status_str.argtypes = [I]
    lib.zk_status_str.restype = ctypes.c_char_p
    lib.zk_ctx_last_error.argtypes = [P]
    lib.zk_ctx_last_error.restype = ctypes.c_char_p
    lib.zk_workspace_bytes.argtypes = [I, I, I]
    lib.zk_workspace_bytes.restype = ctypes.c_size_t
    for f in ("zk_heev_dd", "zk_heev_qd", "zk_heev_dd_allpairs", "zk_heev_dd_noalloc"):
        getattr(lib, f).argtypes = [P, I, ctypes.POINTER(ZkHerm), ctypes.POINTER(ZkEigOut), ctypes.POINTER(ZkOpts)]
    lib.zk_svd_dd.argtypes = [P, I, ctypes.POINTER(ZkMat), ctypes.POINTER(ZkSvdOut), ctypes.POINTER(ZkOpts)]
    lib.zk_mps_create.argtypes = [P, I, I, D, ctypes.POINTER(P)]
    lib.zk_mps_destroy.argtypes = [P]
    lib.zk_mps_apply1.argtypes = [P, I, P]
    lib.zk_mps_apply2.argtypes = [P, I, P, P]
    lib.zk_mps_bond.argtypes = [P, I, I, P, ctypes.POINTER(I)]
    lib.zk_mps_site.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(I), P, ctypes.c_size_t]
    lib.zk_mps_latencies.argtypes = [P, I, P, P, ctypes.POINTER(I)]
    lib.zk_heev_mp.argtypes = [P, I, ctypes.POINTER(ZkHerm), ctypes.POINTER(ZkEigOutMp), ctypes.POINTER(ZkOpts)]
    P2 = P * 2
    lib.zk_mps_two_site_dd.argtypes = [P, I, I, I, P2, P2, P2, I, ctypes.c_double, P2, P2, P2,
                                       ctypes.POINTER(I), ctypes.POINTER(ZkOpts)]
    lib.zk_heev_fp64.argtypes = [P, I, ctypes.POINTER(ZkHerm), ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(I)]
    lib.zk_rqi_refine.argtypes = [P, I, ctypes.POINTER(ZkHerm), I, P, P, I, ctypes.POINTER(ZkEigOut), ctypes.POINTER(ZkOpts)]
    lib.zk_ctx_last_stats.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(ctypes.c_longlong)]
    SZ = ctypes.POINTER(ctypes.c_size_t)
    lib.zk_ctx_memory.argtypes = [P, SZ, SZ, SZ, SZ]
    lib.zk_prof_enable.argtypes = [P, I]
    lib.zk_prof_reset.argtypes = [P]
    lib.zk_prof_classes.argtypes = [P, ctypes.c_uint]
    lib.zk_prof_read.argtypes = [P, I, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(D)]
    if hasattr(lib, "zk_session_create"):
        lib.zk_session_create.argtypes = [P, ctypes.c_size_t, I, ctypes.POINTER(P)]
        lib.zk_session_submit.argtypes = [P, ctypes.POINTER(ZkHerm), ctypes.POINTER(ZkEigOut), I, ctypes.POINTER(ZkOpts),
                                          ctypes.POINTER(ctypes.c_uint64)]
        lib.zk_session_poll.argtypes = [P, ctypes.c_uint64, I, ctypes.POINTER(I)]
        lib.zk_session_times.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)]
        lib.zk_session_destroy.argtypes = [P]
    _lib = lib
    return lib


def status_str(s: int) -> str:
    return load().zk_status_str(int(s)).decode()


def make_opts(tol=0.0, max_iter=0, cluster_tol=0.0, want_vectors=True, init_fp32=False, reorth=True,
              refine=0, shifted_solve=0) -> ZkOpts:
    o = ZkOpts()
    load().zk_opts_default(ctypes.byref(o))
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.cluster_tol = float(cluster_tol)
    o.want_vectors = int(bool(want_vectors))
    o.init_fp32 = int(bool(init_fp32))
    o.reorth = int(bool(reorth))
    o.refine = int(refine)
    o.shifted_solve = int(shifted_solve)
    return o


class Context:
    """A libzk context bound to one device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None, budget: int = 0):
        lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("libzk needs a ROCm GPU; torch.cuda.is_available() is False")
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = lib.zk_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.c_size_t(budget), ctypes.byref(h))
        if rc != ZK_OK:
            raise RuntimeError(f"zk_ctx_create failed: {status_str(rc)}")
        self.handle = h
        self._sessions = []

    def prof(self, on: bool = True):
        load().zk_prof_enable(self.handle, int(bool(on)))

    def prof_reset(self):
        load().zk_prof_reset(self.handle)

    def prof_classes(self, names=None):
        """Time only the named kernel classes (None: all)."""
        mask = 0xFFFFFFFF if names is None else sum(1 << KERNEL_CLASSES.index(n) for n in names)
        load().zk_prof_classes(self.handle, mask)

    def prof_read(self) -> dict:
        """{class name: (total ms, launches, algorithmic work)} of the recorded launches."""
        out = {}
        for c, name in enumerate(KERNEL_CLASSES):
            ms, la, wk = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
            load().zk_prof_read(self.handle, c, ctypes.byref(ms), ctypes.byref(la), ctypes.byref(wk))
            out[name] = (ms.value, la.value, wk.value)
        return out

    def last_error(self) -> str:
        return load().zk_ctx_last_error(self.handle).decode()

    def memory(self) -> dict:
        """Workspace bytes: held now, the budget, the high-water mark, and the
        part held for matrices in flight (zk_ctx_memory)."""
        h, b, hw, tr = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        load().zk_ctx_memory(self.handle, ctypes.byref(h), ctypes.byref(b), ctypes.byref(hw), ctypes.byref(tr))
        return {"held": h.value, "budget": b.value, "high_water": hw.value, "transient": tr.value}

    def last_stats(self) -> dict:
        """Counters of the last heev call's per-pair iteration (zk_ctx_last_stats)."""
        hist = (ctypes.c_int * 16)()
        rounds = ctypes.c_int()
        solves = ctypes.c_longlong()
        load().zk_ctx_last_stats(self.handle, hist, ctypes.byref(rounds), ctypes.byref(solves))
        return {"iters_hist": list(hist), "rounds": rounds.value, "solves": solves.value}

    def close(self):
        # sessions run on this context: stop them first
        for s in getattr(self, "_sessions", []):
            s.close()
        if getattr(self, "handle", None):
            load().zk_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _colmajor(t: torch.Tensor) -> torch.Tensor:
    if t.dtype != torch.complex128 or not t.is_cuda or t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise ValueError("matrices must be square complex128 CUDA tensors")
    return t.transpose(0, 1).contiguous()


def herm(planes, keep: list) -> ZkHerm:
    """ZkHerm for a matrix given as a tensor or a list of limb tensors."""
    if isinstance(planes, torch.Tensor):
        planes = [planes]
    h = ZkHerm()
    n = planes[0].shape[0]
    h.n, h.lda, h.limbs = n, n, len(planes)
    for l, p in enumerate(planes):
        c = _colmajor(p)
        keep.append(c)
        h.plane[l] = c.data_ptr()
    return h


class EigResult:
    """w: (L, n) float64 limbs; V: (L, n, n) complex128 limbs (V[l][:, k] = vector k); info: list of dicts."""

    def __init__(self, w, V, info, status):
        self.w, self.V, self.info, self.status = w, V, info, status

    @property
    def iters(self):
        return [i["iters"] for i in self.info]


def _alloc_out(n: int, L: int, want_vectors: bool, dev, keep: list, npairs: int | None = None):
    k = n if npairs is None else npairs
    o = ZkEigOut()
    o.n, o.ldv, o.limbs = k, n, L
    w = torch.zeros((L, k), dtype=torch.float64, device=dev)
    vbuf = torch.zeros((L, k, n), dtype=torch.complex128, device=dev) if want_vectors else None
    for l in range(L):
        o.w[l] = w[l].data_ptr()
        o.v[l] = vbuf[l].data_ptr() if vbuf is not None else None
    info = (ZkPairInfo * k)()
    o.info = ctypes.cast(info, ctypes.POINTER(ZkPairInfo))
    keep += [w, vbuf, info]
    V = vbuf.transpose(1, 2) if vbuf is not None else None
    return o, w, V, info


def _info_list(info, k):
    return [{"iters": info[i].iters, "flags": info[i].flags, "cluster": info[i].cluster, "resid": info[i].resid}
            for i in range(k)]


def heev(ctx: Context, mats, limbs_out: int = 2, opts: ZkOpts | None = None, stats: dict | None = None,
         noalloc: bool = False):
    """Eigendecompose a list of matrices (each a tensor or list of limb tensors).

    noalloc=True (double-double only) calls zk_heev_dd_noalloc, whose
    workspace is the library's static scratch array instead of the context's.
    Returns a list of EigResult (status is shared by the batch call).
    """
    if noalloc and limbs_out != 2:
        raise ValueError("the no-allocation entry point gives double-double output only")
    lib = load()
    keep: list = []
    count = len(mats)
    H = (ZkHerm * count)()
    O = (ZkEigOut * count)()
    outs = []
    want = True if opts is None else bool(opts.want_vectors)
    for i, m in enumerate(mats):
        H[i] = herm(m, keep)
        o, w, V, info = _alloc_out(H[i].n, limbs_out, want, ctx_device(m), keep)
        O[i] = o
        outs.append((w, V, info, H[i].n))
    op = ctypes.byref(opts) if opts is not None else None
    f = (lib.zk_heev_dd_noalloc if noalloc else lib.zk_heev_dd) if limbs_out == 2 else lib.zk_heev_qd
    rc = f(ctx.handle, count, H, O, op)
    if stats is not None:
        stats.update(ctx.last_stats())
    if rc not in (ZK_OK, ZK_ENOCONV):
        raise RuntimeError(f"zk_heev failed: {status_str(rc)}: {ctx.last_error()}")
    return [EigResult(w, V, _info_list(info, n), rc) for (w, V, info, n) in outs]


def heev_allpairs(ctx: Context, mats, opts: ZkOpts | None = None):
    """Double-double eigendecomposition with the all-pairs refinement
    (zk_heev_dd_allpairs) in place of the per-pair Rayleigh quotient
    iteration.  Same inputs and results as heev(..., limbs_out=2)."""
    lib = load()
    keep: list = []
    count = len(mats)
    H = (ZkHerm * count)()
    O = (ZkEigOut * count)()
    outs = []
    want = True if opts is None else bool(opts.want_vectors)
    for i, m in enumerate(mats):
        H[i] = herm(m, keep)
        o, w, V, info = _alloc_out(H[i].n, 2, want, ctx_device(m), keep)
        O[i] = o
        outs.append((w, V, info, H[i].n))
    op = ctypes.byref(opts) if opts is not None else None
    rc = lib.zk_heev_dd_allpairs(ctx.handle, count, H, O, op)
    if rc not in (ZK_OK, ZK_ENOCONV):
        raise RuntimeError(f"zk_heev_dd_allpairs failed: {status_str(rc)}: {ctx.last_error()}")
    return [EigResult(w, V, _info_list(info, n), rc) for (w, V, info, n) in outs]


def heev_mp(ctx: Context, mats, limbs: int = 8, opts: ZkOpts | None = None):
    """Eigendecomposition to `limbs` (4, 8 or 16) binary64 limbs per value
    (zk_heev_mp): w (limbs, n), V (limbs, n, n) with V[l][:, k] limb l of
    eigenvector k."""
    lib = load()
    keep: list = []
    count = len(mats)
    H = (ZkHerm * count)()
    O = (ZkEigOutMp * count)()
    outs = []
    want = True if opts is None else bool(opts.want_vectors)
    for i, m in enumerate(mats):
        H[i] = herm(m, keep)
        n = H[i].n
        w = torch.zeros((limbs, n), dtype=torch.float64, device=ctx_device(m))
        vb = torch.zeros((limbs, n, n), dtype=torch.complex128, device=ctx_device(m)) if want else None
        info = (ZkPairInfo * n)()
        O[i].n, O[i].ldv, O[i].limbs = n, n, limbs
        O[i].w = w.data_ptr()
        O[i].v = vb.data_ptr() if vb is not None else None
        O[i].info = ctypes.cast(info, ctypes.POINTER(ZkPairInfo))
        keep += [w, vb, info]
        outs.append((w, vb.transpose(1, 2) if vb is not None else None, info, n))
    op = ctypes.byref(opts) if opts is not None else None
    rc = lib.zk_heev_mp(ctx.handle, count, H, O, op)
    if rc not in (ZK_OK, ZK_ENOCONV):
        raise RuntimeError(f"zk_heev_mp failed: {status_str(rc)}: {ctx.last_error()}")
    return [EigResult(w, V, _info_list(info, n), rc) for (w, V, info, n) in outs]


def _gate_planes(G, dim):
    """Two limb planes (hi, lo) of a dim x dim complex gate, column-major, as
    one float64 array: G is a complex array or a pair of them (limbs)."""
    limbs = list(G) if isinstance(G, (list, tuple)) else [np.asarray(G, dtype=np.complex128), None]
    if len(limbs) == 1:
        limbs.append(None)
    out = np.zeros(2 * 2 * dim * dim, dtype=np.float64)
    for p, g in enumerate(limbs[:2]):
        if g is None:
            continue
        g = np.asarray(g, dtype=np.complex128)
        if g.shape != (dim, dim):
            raise ValueError(f"gate must be {dim} x {dim}")
        out[p * 2 * dim * dim:(p + 1) * 2 * dim * dim] = np.ascontiguousarray(g.T).view(np.float64).ravel()
    return out


class Mps:
    """A chain of qubits as a double-double matrix product state (zk_mps_*):
    two-qubit gates emit Hermitian bond matrices that a serving session
    eigendecomposes, one layer of disjoint gates at a time."""

    def __init__(self, ctx: Context, nq: int, chi_max: int = 64, cutoff: float = 0.0):
        self.lib = load()
        self.ctx = ctx
        self.nq = nq
        h = ctypes.c_void_p()
        rc = self.lib.zk_mps_create(ctx.handle, nq, chi_max, float(cutoff), ctypes.byref(h))
        if rc != ZK_OK:
            raise RuntimeError(f"zk_mps_create failed: {status_str(rc)}: {ctx.last_error()}")
        self.handle = h

    def apply1(self, q: int, G):
        g = _gate_planes(G, 2)
        rc = self.lib.zk_mps_apply1(self.handle, q, g.ctypes.data)
        if rc != ZK_OK:
            raise RuntimeError(f"zk_mps_apply1 failed: {status_str(rc)}: {self.ctx.last_error()}")

    def apply2(self, qs, gates) -> int:
        """Gates on the disjoint pairs (q, q+1) for q in qs; returns the status."""
        arrs = [_gate_planes(G, 4) for G in gates]
        ptrs = (ctypes.c_void_p * max(1, len(arrs)))(*[a.ctypes.data for a in arrs])
        qa = (ctypes.c_int * max(1, len(qs)))(*qs)
        rc = self.lib.zk_mps_apply2(self.handle, len(qs), qa, ptrs)
        if rc not in (ZK_OK, ZK_ENOCONV):
            raise RuntimeError(f"zk_mps_apply2 failed: {status_str(rc)}: {self.ctx.last_error()}")
        return rc

    def bond(self, b: int) -> np.ndarray:
        """(2, chi) limbs of the squared Schmidt values of bond b, descending."""
        chi = ctypes.c_int()
        self.lib.zk_mps_bond(self.handle, b, 0, None, ctypes.byref(chi))
        out = np.zeros(2 * chi.value, dtype=np.float64)
        rc = self.lib.zk_mps_bond(self.handle, b, chi.value, out.ctypes.data, ctypes.byref(chi))
        if rc != ZK_OK:
            raise RuntimeError(f"zk_mps_bond failed: {status_str(rc)}")
        return out.reshape(2, chi.value)

    def site(self, q: int):
        """(2, chi_l, 2, chi_r) complex limbs of B_q[l, s, r]."""
        cl, cr = ctypes.c_int(), ctypes.c_int()
        self.lib.zk_mps_site(self.handle, q, ctypes.byref(cl), ctypes.byref(cr), None, 0)
        n = 2 * cl.value * 2 * cr.value
        out = np.zeros(2 * n, dtype=np.float64)
        rc = self.lib.zk_mps_site(self.handle, q, ctypes.byref(cl), ctypes.byref(cr), out.ctypes.data, out.size)
        if rc != ZK_OK:
            raise RuntimeError(f"zk_mps_site failed: {status_str(rc)}")
        z = out.view(np.complex128).reshape(2, 2 * cr.value, cl.value)   # plane, column (s r), row l
        return np.ascontiguousarray(z.reshape(2, 2, cr.value, cl.value).transpose(0, 3, 1, 2))

    def latencies(self):
        """(seconds, orders) of every bond matrix diagonalised so far."""
        cnt = ctypes.c_int()
        self.lib.zk_mps_latencies(self.handle, 0, None, None, ctypes.byref(cnt))
        sec = np.zeros(max(1, cnt.value))
        ords = np.zeros(max(1, cnt.value), dtype=np.int32)
        self.lib.zk_mps_latencies(self.handle, cnt.value, sec.ctypes.data, ords.ctypes.data, ctypes.byref(cnt))
        return sec[:cnt.value], ords[:cnt.value]

    def close(self):
        if getattr(self, "handle", None):
            self.lib.zk_mps_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SvdResult:
    """s: (2, k) float64 limbs (descending); U: (2, m, k), V: (2, n, k) complex128 limbs; info: list of dicts."""

    def __init__(self, s, U, V, info, status):
        self.s, self.U, self.V, self.info, self.status = s, U, V, info, status


def svd(ctx: Context, mats, opts: ZkOpts | None = None):
    """Double-double singular value decomposition (zk_svd_dd) of a list of
    general matrices, each an (m, n) tensor or a list of limb tensors."""
    lib = load()
    keep: list = []
    count = len(mats)
    A = (ZkMat * count)()
    O = (ZkSvdOut * count)()
    outs = []
    want = True if opts is None else bool(opts.want_vectors)
    for i, mat in enumerate(mats):
        planes = [mat] if isinstance(mat, torch.Tensor) else list(mat)
        m, n = planes[0].shape
        dev = planes[0].device
        A[i].m, A[i].n, A[i].lda, A[i].limbs = m, n, m, len(planes)
        for l, p in enumerate(planes):
            if p.dtype != torch.complex128 or not p.is_cuda or p.dim() != 2 or tuple(p.shape) != (m, n):
                raise ValueError("matrices must be complex128 CUDA tensors of one shape per matrix")
            c = p.transpose(0, 1).contiguous()   # column-major storage
            keep.append(c)
            A[i].plane[l] = c.data_ptr()
        k = min(m, n)
        s = torch.zeros((2, k), dtype=torch.float64, device=dev)
        ub = torch.zeros((2, k, m), dtype=torch.complex128, device=dev) if want else None
        vb = torch.zeros((2, k, n), dtype=torch.complex128, device=dev) if want else None
        o = O[i]
        o.m, o.n, o.limbs, o.ldu, o.ldv = m, n, 2, m, n
        for l in range(2):
            o.s[l] = s[l].data_ptr()
            o.u[l] = ub[l].data_ptr() if want else None
            o.v[l] = vb[l].data_ptr() if want else None
        info = (ZkPairInfo * k)()
        o.info = ctypes.cast(info, ctypes.POINTER(ZkPairInfo))
        keep += [s, ub, vb, info]
        outs.append((s, ub.transpose(1, 2) if want else None, vb.transpose(1, 2) if want else None, info, k))
    op = ctypes.byref(opts) if opts is not None else None
    rc = lib.zk_svd_dd(ctx.handle, count, A, O, op)
    if rc not in (ZK_OK, ZK_ENOCONV):
        raise RuntimeError(f"zk_svd_dd failed: {status_str(rc)}: {ctx.last_error()}")
    return [SvdResult(s, U, V, _info_list(info, k), rc) for (s, U, V, info, k) in outs]


class MpsResult:
    """A: (2, 2 chi_l, chi') and B: (2, chi', 2 chi_r) complex128 limbs, s: (2, chi') float64 limbs."""

    def __init__(self, A, s, B, chi, status):
        self.A, self.s, self.B, self.chi, self.status = A, s, B, chi, status


def _limb_pair(x):
    """Two complex128 limb tensors (hi, lo) from a tensor or a list of one or two."""
    planes = [x] if isinstance(x, torch.Tensor) else list(x)
    if len(planes) == 1:
        planes = planes + [torch.zeros_like(planes[0])]
    if len(planes) != 2:
        raise ValueError("expected one or two limb tensors")
    for p in planes:
        if p.dtype != torch.complex128 or not p.is_cuda or p.dim() != 2 or p.shape != planes[0].shape:
            raise ValueError("limbs must be complex128 CUDA matrices of one shape")
    return planes


def mps_two_site(ctx: Context, A, B, gate, chi_max: int, cutoff: float = 0.0, opts: ZkOpts | None = None):
    """One double-double two-site update (zk_mps_two_site_dd).

    A: (2 chi_l, chi) with row index s1 chi_l + l; B: (chi, 2 chi_r) with
    column index s2 chi_r + r; gate: (4, 4) with index 2 s1 + s2; each a
    complex128 CUDA tensor or a list of (hi, lo) limb tensors."""
    lib = load()
    Ap, Bp, Gp = _limb_pair(A), _limb_pair(B), _limb_pair(gate)
    M, chi = Ap[0].shape
    chi2, N = Bp[0].shape
    if chi2 != chi or M % 2 or N % 2 or tuple(Gp[0].shape) != (4, 4):
        raise ValueError("shapes: A (2 chi_l, chi), B (chi, 2 chi_r), gate (4, 4)")
    keep = [p.transpose(0, 1).contiguous() for p in Ap + Bp + Gp]   # column-major storage
    dev = Ap[0].device
    Ao = [torch.zeros((chi_max, M), dtype=torch.complex128, device=dev) for _ in range(2)]
    Bo = [torch.zeros((chi_max * N,), dtype=torch.complex128, device=dev) for _ in range(2)]
    so = [torch.zeros((chi_max,), dtype=torch.float64, device=dev) for _ in range(2)]
    P2 = ctypes.c_void_p * 2
    chi_out = ctypes.c_int(0)
    torch.cuda.current_stream().synchronize()
    rc = lib.zk_mps_two_site_dd(ctx.handle, M // 2, chi, N // 2, P2(keep[0].data_ptr(), keep[1].data_ptr()),
                                P2(keep[2].data_ptr(), keep[3].data_ptr()), P2(keep[4].data_ptr(), keep[5].data_ptr()),
                                chi_max, float(cutoff), P2(Ao[0].data_ptr(), Ao[1].data_ptr()),
                                P2(Bo[0].data_ptr(), Bo[1].data_ptr()), P2(so[0].data_ptr(), so[1].data_ptr()),
                                ctypes.byref(chi_out), ctypes.byref(opts) if opts is not None else None)
    if rc not in (ZK_OK, ZK_ENOCONV):
        raise RuntimeError(f"zk_mps_two_site_dd failed: {status_str(rc)}: {ctx.last_error()}")
    c = chi_out.value
    A_new = torch.stack([a[:c].transpose(0, 1) for a in Ao])
    B_new = torch.stack([b[:c * N].reshape(N, c).transpose(0, 1) for b in Bo])
    s_new = torch.stack([x[:c] for x in so])
    return MpsResult(A_new, s_new, B_new, c, rc)


def ctx_device(m):
    t = m if isinstance(m, torch.Tensor) else m[0]
    return t.device


def heev_fp64(ctx: Context, mats):
    """Stage 1 alone: list of (w (n,), V (n, n)) binary64 eigenpairs."""
    lib = load()
    keep: list = []
    count = len(mats)
    H = (ZkHerm * count)()
    W = (ctypes.c_void_p * count)()
    Vp = (ctypes.c_void_p * count)()
    ld = (ctypes.c_int * count)()
    res = []
    for i, m in enumerate(mats):
        H[i] = herm(m, keep)
        n = H[i].n
        w = torch.zeros(n, dtype=torch.float64, device=ctx_device(m))
        vb = torch.zeros((n, n), dtype=torch.complex128, device=ctx_device(m))
        W[i], Vp[i], ld[i] = w.data_ptr(), vb.data_ptr(), n
        res.append((w, vb.transpose(0, 1)))
        keep += [w, vb]
    rc = lib.zk_heev_fp64(ctx.handle, count, H, W, Vp, ld)
    if rc != ZK_OK:
        raise RuntimeError(f"zk_heev_fp64 failed: {status_str(rc)}: {ctx.last_error()}")
    return res


def rqi_refine(ctx: Context, planes, w0: torch.Tensor, V0: torch.Tensor, limbs_out: int = 2, opts: ZkOpts | None = None):
    """Stage 2 alone on caller binary64 pairs: w0 (k,), V0 (n, k) (columns = vectors)."""
    lib = load()
    keep: list = []
    h = herm(planes, keep)
    n = h.n
    k = int(w0.shape[0])
    w0c = w0.to(torch.float64).contiguous()
    V0c = V0.transpose(0, 1).contiguous()   # row j = vector j -> column-major n x k, ld n
    keep += [w0c, V0c]
    want = True if opts is None else bool(opts.want_vectors)
    o, w, V, info = _alloc_out(n, limbs_out, want, w0.device, keep, npairs=k)
    rc = lib.zk_rqi_refine(ctx.handle, limbs_out, ctypes.byref(h), k, ctypes.c_void_p(w0c.data_ptr()),
                           ctypes.c_void_p(V0c.data_ptr()), n, ctypes.byref(o),
                           ctypes.byref(opts) if opts is not None else None)
    if rc not in (ZK_OK, ZK_ENOCONV):
        raise RuntimeError(f"zk_rqi_refine failed: {status_str(rc)}: {ctx.last_error()}")
    return EigResult(w, V, _info_list(info, k), rc)


class Session:
    """Serving session (continuous batching) on a context; see zk_session_* in zk.h."""

    def __init__(self, ctx: Context, budget: int = 0, max_queue: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        rc = lib.zk_session_create(ctx.handle, ctypes.c_size_t(budget), int(max_queue), ctypes.byref(h))
        if rc != ZK_OK:
            raise RuntimeError(f"zk_session_create failed: {status_str(rc)}")
        self.ctx = ctx
        self.handle = h
        self._req = {}
        ctx._sessions.append(self)

    def submit(self, planes, limbs_out: int = 2, opts: ZkOpts | None = None) -> int:
        """Queue a request; returns its ticket.  Raises on ZK_EINVAL / ZK_ENOMEM / ZK_EAGAIN."""
        lib = load()
        keep: list = []
        h = herm(planes, keep)
        want = True if opts is None else bool(opts.want_vectors)
        o, w, V, info = _alloc_out(h.n, limbs_out, want, ctx_device(planes), keep)
        t = ctypes.c_uint64()
        # the column-major copies and outputs must be complete before the scheduler reads them
        torch.cuda.current_stream().synchronize()
        rc = lib.zk_session_submit(self.handle, ctypes.byref(h), ctypes.byref(o), limbs_out,
                                   ctypes.byref(opts) if opts is not None else None, ctypes.byref(t))
        if rc != ZK_OK:
            raise RuntimeError(f"zk_session_submit: {status_str(rc)}")
        self._req[t.value] = (keep, w, V, info, h.n, o, h)
        return t.value

    def poll(self, ticket: int, timeout_us: int = -1):
        """(rc, request status): rc ZK_OK when done, ZK_EAGAIN while pending."""
        st = ctypes.c_int()
        rc = load().zk_session_poll(self.handle, ctypes.c_uint64(ticket), int(timeout_us), ctypes.byref(st))
        return rc, st.value

    def times(self, ticket: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        load().zk_session_times(self.handle, ctypes.c_uint64(ticket), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return a.value, b.value, c.value

    def result(self, ticket: int) -> EigResult:
        rc, status = self.poll(ticket, -1)
        if rc != ZK_OK:
            raise RuntimeError(f"request {ticket}: {status_str(rc)}")
        keep, w, V, info, n, o, h = self._req[ticket]
        return EigResult(w, V, _info_list(info, n), status)

    def close(self):
        if getattr(self, "handle", None):
            load().zk_session_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
