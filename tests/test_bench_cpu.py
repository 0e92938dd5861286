"""Host-side logic of bench.py (no GPU): the phase-rate arithmetic, the source-hash guard
on the committed counter summaries, and the one-GPU refusal."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_phase_rooflines_counts():
    n, N, L = 4096, 64, 64
    tm = {"assemble_ms": 6.0, "solve_ms": 26.0, "residual_ms": 31.0}
    out = bench.phase_rooflines(n, N, L, tm, iters=2)
    n2 = float(n) * n
    # the assembly writes a c64 and a c128 copy of every T(z_k)
    assert out["assembly"]["bytes"] == N * 24 * n2
    assert out["assembly"]["GB_s"] == pytest.approx(N * 24 * n2 / 6e-3 / 1e9, rel=1e-3)
    # one solve and one FP64 residual before refinement, then one of each per correction
    assert out["solves"]["passes"] == 3 and out["residual"]["passes"] == 3
    assert out["solves"]["flops"] == 3 * N * 8 * n2 * L
    assert out["solves"]["bytes"] == 3 * N * 8 * n2
    assert out["residual"]["bytes"] == 3 * N * 16 * n2
    assert out["residual"]["fp64_mfma_frac"] == pytest.approx(
        3 * N * 8 * n2 * L / 31e-3 / 1e12 / bench.PEAK_FP64_MFMA_TFLOPS, rel=1e-3)
    # a phase that was not timed is left out
    assert "assembly" not in bench.phase_rooflines(n, N, L, {"solve_ms": 1.0}, iters=0)


def _copy_tree(tmp_path):
    for d in ("profiles", os.path.join("paper_1605_07951_amd", "csrc")):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d)
    return tmp_path


def test_counter_figures_follow_the_sources(tmp_path, monkeypatch):
    # the committed summaries match the committed kernels
    assert isinstance(bench.measured_traffic(), int) and bench.measured_traffic() > 0
    assert 0.0 < bench.measured_mfma_util() <= 1.0
    # a change to the update kernel's source voids both figures
    root = _copy_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic() is not None
    with open(root / "paper_1605_07951_amd" / "csrc" / "gemm.hip", "a") as f:
        f.write("\n// edited\n")
    assert bench.measured_traffic() is None
    assert bench.measured_mfma_util() is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus_requested"] == 2 and "one GPU" in msg["error"]
