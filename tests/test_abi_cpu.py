"""The C-ABI library loads and exports every function include/zk.h declares (no GPU needed)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zk.h")
LIB = os.path.join(ROOT, "paper_2402_11868_amd", "libzk.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(zk_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("zk_heev_dd", "zk_heev_qd", "zk_rqi_refine", "zk_session_submit", "zk_session_poll",
              "zk_ctx_create", "zk_heev_fp64", "zk_heev_dd_allpairs", "zk_svd_dd", "zk_mps_two_site_dd"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        import paper_2402_11868_amd.build as b   # build step only; no device code runs
        b.build()
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    for n in declared():
        assert re.search(rf"\bT {n}\b", out), n


def test_static_entry_points_without_device():
    lib = ctypes.CDLL(LIB)
    lib.zk_status_str.restype = ctypes.c_char_p
    assert lib.zk_status_str(0) == b"ZK_OK"
    assert lib.zk_status_str(-1).startswith(b"ZK_EINVAL")
    lib.zk_workspace_bytes.restype = ctypes.c_size_t
    assert lib.zk_workspace_bytes(1024, 2, 4) > 4 * 1024 * 1025 * 32
    assert lib.zk_workspace_bytes(0, 2, 1) == 0
    # NULL handles are rejected before any device work
    assert lib.zk_heev_dd(None, 1, None, None, None) == -1
    assert lib.zk_heev_dd_allpairs(None, 1, None, None, None) == -1
    assert lib.zk_heev_dd_noalloc(None, 1, None, None, None) == -1
    assert lib.zk_svd_dd(None, 1, None, None, None) == -1
    assert lib.zk_mps_two_site_dd(None, 1, 1, 1, None, None, None, 1, ctypes.c_double(0.0), None, None, None,
                                  None, None) == -1
    assert lib.zk_session_submit(None, None, None, 2, None, None) == -1
    assert lib.zk_ctx_destroy(None) == 0


def test_context_queries_reject_null():
    lib = ctypes.CDLL(LIB)
    assert lib.zk_ctx_memory(None, None, None, None, None) == -1
    assert lib.zk_ctx_last_stats(None, None, None, None) == -1
