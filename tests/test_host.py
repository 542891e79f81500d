"""CPU checks of host-side behaviour: the binding refuses to run without the
HIP library (there is no fallback), and the benchmark's argument handling and
context figures."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_missing_library_raises(monkeypatch, tmp_path):
    from paper_2308_16317_amd import lsms

    monkeypatch.setattr(lsms, "_lib", None)
    monkeypatch.setattr(lsms, "LIB_PATH", str(tmp_path / "liblsms_tau.so"))
    with pytest.raises(RuntimeError, match="missing"):
        lsms.lib()


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_bench_refuses_several_gpus():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_bench_refuses_precision_form_in_chunked_mode():
    r = _bench("--precision", "fp32ir", "--mode", "chunked")
    assert r.returncode == 2
    assert "tau00_solve" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_paper_speedups_match_their_wall_clock_times():
    # Sec. 4.2, table of performance results: GPU and CPU wall-clock seconds
    sys.path.insert(0, ROOT)
    import bench

    assert len(bench.PAPER_SPEEDUPS) == 5
    for row in bench.PAPER_SPEEDUPS:
        gpu_s, cpu_s = row["seconds"]
        assert row["speedup"] == pytest.approx(cpu_s / gpu_s, rel=5e-3), row
        assert "EPYC 7742" in row["cpu"] and ("A100" in row["gpu"] or "V100" in row["gpu"])


def test_kernel_hash_ignores_comments_only(tmp_path):
    import shutil

    sys.path.insert(0, ROOT)
    import bench

    csrc = os.path.join(ROOT, "paper_2308_16317_amd", "csrc")
    for f in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(csrc, f), tmp_path / f)
    h0 = bench.kernel_source_hash(str(tmp_path))
    assert h0 == bench.kernel_source_hash()
    p = tmp_path / "lu_device.h"
    src = p.read_text()
    p.write_text("// a new comment line\n" + src.replace("\n", "  \n", 3) + "/* block\ncomment */\n")
    assert bench.kernel_source_hash(str(tmp_path)) == h0
    p.write_text(src + "\nstatic int extra_symbol;\n")
    assert bench.kernel_source_hash(str(tmp_path)) != h0
