"""Host logic of bench.py (no GPU): the completion kernel's source digest,
the HBM traffic record it keys, and the one-GPU contract."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

SOURCES = ("kernels_adm.hip", "adm_common.h", "vplmc_internal.h")


@pytest.fixture
def tree(tmp_path, monkeypatch):
    """A copy of the digested sources and the traffic record under a temporary root."""
    csrc = tmp_path / "paper_2202_12567_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2202_12567_amd", "csrc", f), csrc / f)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def edit(tree, f, fn):
    p = tree / "paper_2202_12567_amd" / "csrc" / f
    p.write_text(fn(p.read_text()))


def test_digest_ignores_comments_and_blank_lines(tree):
    d0 = bench.source_digest()
    edit(tree, "kernels_adm.hip", lambda s: "// a new leading comment\n\n" + s.replace("\n", "  // note\n", 3))
    assert bench.source_digest() == d0


def test_digest_follows_code(tree):
    d0 = bench.source_digest()
    edit(tree, "kernels_adm.hip", lambda s: s.replace("constexpr int ADM_CMB = 4;", "constexpr int ADM_CMB = 5;"))
    assert bench.source_digest() != d0
    edit(tree, "kernels_adm.hip", lambda s: s.replace("constexpr int ADM_CMB = 5;", "constexpr int ADM_CMB = 4;"))
    assert bench.source_digest() == d0
    edit(tree, "adm_common.h", lambda s: s.replace("constexpr int GRAM_STAGE = 16384;", "constexpr int GRAM_STAGE = 8192;"))
    d1 = bench.source_digest()
    assert d1 != d0
    edit(tree, "vplmc_internal.h", lambda s: s + "\nconstexpr int UNUSED_FOR_THE_TEST = 1;\n")
    assert bench.source_digest() not in (d0, d1)


def test_traffic_record_is_keyed_by_rate_and_source(tree):
    rec = {"ppm": 25000, "source_sha256": bench.source_digest(), "bytes_per_launch": 123456789,
           "coarsen": "32768:512", "rank": 16}
    path = tree / "profiles" / "k_adm_ell_mid_traffic.json"
    for p in (tree / "profiles").glob("k_adm_ell_*_traffic.json"):
        p.unlink()
    assert bench.measured_traffic("mid", 25000, "32768:512", 16) is None          # no record
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("mid", 25000, "32768:512", 16) == 123456789
    assert bench.measured_traffic("mid", 2500, "32768:512", 16) is None           # other rate
    assert bench.measured_traffic("frame", 25000, "32768:512", 16) is None        # other workload
    assert bench.measured_traffic("mid", 25000, "none", 0) is None                # other coarsening
    assert bench.measured_traffic("mid", 25000, "32768:512", 8) is None           # other rank
    edit(tree, "kernels_adm.hip", lambda s: s + "\nconstexpr int UNUSED_FOR_THE_TEST = 1;\n")
    assert bench.measured_traffic("mid", 25000, "32768:512", 16) is None          # other code


def test_committed_traffic_records_match_the_committed_kernel():
    import glob
    paths = glob.glob(os.path.join(ROOT, "profiles", "k_adm_ell_*_traffic.json"))
    assert paths, "the benchmark's traffic record is committed"
    for path in paths:
        with open(path) as fh:
            rec = json.load(fh)
        assert rec["source_sha256"] == bench.source_digest(), path
        assert rec["bytes_per_launch"] == rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
