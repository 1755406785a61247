"""Host-side checks of bench.py's bookkeeping (no GPU): the digest that keys
the stored HBM traffic of the trailing update finds every region it hashes,
changes when the update kernel's section changes and not when another
kernel of the same file does, and the stored profile parses."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_digest_regions_present():
    d = bench.kernel_source_digest()
    assert len(d) == 64


def test_digest_tracks_the_update_section_only(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_2402_11868_amd", "csrc", "stage2.hip")
    text = open(src).read()
    base = bench.kernel_source_digest()
    copy = tmp_path / "stage2.hip"

    def digest_of(t):
        copy.write_text(t)
        regions = [(str(copy), b, e) for _, b, e in bench.LU_UPDATE_REGIONS]
        monkeypatch.setattr(bench, "LU_UPDATE_REGIONS", regions)
        monkeypatch.setattr(bench, "ROOT", ROOT)
        return bench.kernel_source_digest()

    assert digest_of(text) == base
    # a change inside the update kernel's section
    marker = "const bool diag = LDL && ti == tj;"
    assert marker in text
    assert digest_of(text.replace(marker, marker + " ", 1)) != base
    # a change in another kernel of the file (the Gram-Schmidt Cholesky)
    other = "k_gs_chol(const GsCluster *cls"
    assert other in text
    assert digest_of(text.replace(other, other + " ", 1)) == base


def test_stored_traffic_file_parses():
    path = os.path.join(ROOT, bench.TRAFFIC_FILE)
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    assert len(kv["kernel_source_sha256"]) == 64
    assert float(kv["traffic_bytes_per_launch"]) > 0
