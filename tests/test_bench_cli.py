"""bench.py on the host: one GPU only (several GPUs exit with a message and
status 2, before anything is built or touches a GPU), and the HBM traffic
records it reports apply only while the kernel's source has the hash they
were taken on."""

import os
import subprocess
import sys

from conftest import ROOT


def test_several_gpus_are_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_records_follow_the_kernel_source(tmp_path, monkeypatch):
    import hashlib
    sys.path.insert(0, ROOT)
    import bench
    src = tmp_path / "paper_1708_02845_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "gemm.hip").write_bytes(b"kernel source v1")
    sha = hashlib.sha1(b"kernel source v1").hexdigest()[:12]
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "hbm_traffic.txt").write_text(
        "# comment\n"
        f"grid1025_T64 kl_gemm_f16x3 1000 24 {sha}\n"
        "grid1025_T64 kl_gemm_f16x3 5 5 000000000000\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("grid1025_T64", "kl_gemm_f16x3") == 1024
    assert bench.measured_traffic("grid257", "kl_gemm_f16x3") is None
    assert bench.measured_traffic("grid1025", "no_such_kernel") is None
    # the source changes: the record no longer applies
    (src / "gemm.hip").write_bytes(b"kernel source v2")
    assert bench.measured_traffic("grid1025_T64", "kl_gemm_f16x3") is None
