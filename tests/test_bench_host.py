"""Host logic of bench.py that runs without a GPU: the one-GPU guard and the
reading of the committed HBM-counter summary (used only while it was taken on
the current kernel source)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def _tree(tmp_path, body, sha_line):
    src = tmp_path / "paper_2408_06698_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "kernels.hip").write_text("namespace hopu {\n" + body + "\n// " + "-" * 66 + " launchers\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.txt").write_text(f"# header = ignored\n{sha_line}\nmass_bytes_per_launch = 12345\n")


def test_traffic_read_only_for_the_profiled_source(tmp_path, monkeypatch):
    from paper_2408_06698_amd.rocpd_summary import kernels_sha
    _tree(tmp_path, "int a;", "kernels_sha = 0000000000000000")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profiles("mass") is None          # taken on other source
    sha = kernels_sha(str(tmp_path / "paper_2408_06698_amd" / "csrc" / "kernels.hip"))
    (tmp_path / "profiles" / "traffic.txt").write_text(f"kernels_sha = {sha}\nmass_bytes_per_launch = 12345\n")
    assert bench.traffic_from_profiles("mass") == pytest.approx(12345.0)
    assert bench.traffic_from_profiles("elem") is None          # no such key
    (tmp_path / "profiles" / "traffic.txt").unlink()
    assert bench.traffic_from_profiles("mass") is None          # no summary


def test_traffic_of_other_sources_ignores_comment_edits(tmp_path, monkeypatch):
    """Sources other than kernels.hip are keyed by their code without //
    comments and blank lines: a comment edit keeps the recorded traffic, a
    code edit drops it."""
    from paper_2408_06698_amd.rocpd_summary import source_sha
    src = tmp_path / "paper_2408_06698_amd" / "csrc"
    src.mkdir(parents=True)
    code = "__global__ void k(double* y) {  // one\n  y[0] = 1.0;\n}\n"
    (src / "other.hip").write_text(code)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "x_traffic.txt").write_text(f"kernels_sha = {source_sha(code)}\nk_bytes_per_launch = 777\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profiles("k", "other.hip") == pytest.approx(777.0)
    (src / "other.hip").write_text("// a new header comment\n\n" + code.replace("// one", "// two"))
    assert bench.traffic_from_profiles("k", "other.hip") == pytest.approx(777.0)
    (src / "other.hip").write_text(code.replace("1.0", "2.0"))
    assert bench.traffic_from_profiles("k", "other.hip") is None

