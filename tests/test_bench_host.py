"""Host logic of bench.py (CPU): the one-GPU rule, the counter summary that
feeds roofline.traffic (read only while the sweep's sources are unchanged,
comments aside) and the oracle baseline's record."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import problems as P  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def _sources(tmp_path, body):
    p = tmp_path / "k.hip"
    p.write_text(body)
    return [str(p)]


def test_source_digest_ignores_comments_only(tmp_path, monkeypatch):
    code = "int f(int x) {\n  return x + 1;\n}\n"
    monkeypatch.setattr(bench, "SWEEP_SOURCES", _sources(tmp_path, code))
    d0 = bench.sweep_source_digest()
    commented = "// the increment\nint f(int x) {  // one\n\n  return x + 1;  /* add\n  one */\n}\n"
    monkeypatch.setattr(bench, "SWEEP_SOURCES", _sources(tmp_path, commented))
    assert bench.sweep_source_digest() == d0
    monkeypatch.setattr(bench, "SWEEP_SOURCES", _sources(tmp_path, code.replace("1", "2")))
    assert bench.sweep_source_digest() != d0


def test_traffic_is_read_only_for_the_profiled_sources_and_kernel(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "SWEEP_SOURCES", _sources(tmp_path, "int k;\n"))
    digest = bench.sweep_source_digest()
    f = tmp_path / "traffic.txt"

    def write(sha, kernel="k_sweep<2, 2, false, true, true>"):
        f.write_text("# FETCH_SIZE 1 KiB: not a field\n"
                     f"kernel: {kernel}\nsweep_source_sha256: {sha}\n"
                     "hbm_bytes_per_launch: 7.895213e+10\n")

    write(digest)
    assert bench.measured_traffic(str(f)) == pytest.approx(7.895213e10)
    write("0" * 64)
    assert bench.measured_traffic(str(f)) is None
    write(digest, kernel="k_sweep<3, 1, false, true, true>")
    assert bench.measured_traffic(str(f)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.txt")) is None


def test_committed_counter_summaries_name_their_kernels():
    for path, kernel in ((bench.TRAFFIC_FILE, bench.SWEEP_KERNEL),
                         (bench.TRAFFIC_FILE_3D, "k_sweep<3, 1, false, true, true>")):
        fields = dict(ln.split(":", 1) for ln in open(path) if ":" in ln and not ln.startswith("#"))
        assert fields["kernel"].strip() == kernel
        assert len(fields["sweep_source_sha256"].strip()) == 64
        assert float(fields["hbm_bytes_per_launch"]) > 0


def test_oracle_baseline_record():
    pr = P.config_c1()
    r = bench.cpu_baseline(pr, 4, 0.01)
    assert r["kind"] == "oracle" and r["extrapolated"] and r["unit"] == "unknowns/s"
    assert 1 <= r["cores"] <= 16 and r["value"] > 0
    assert "4 sampled velocities" in r["sample"]
