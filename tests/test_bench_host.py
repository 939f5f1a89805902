"""Host checks of bench.py (no GPU): the one-GPU refusal, the algorithmic byte counts the
roofline divides by, and the ALU peaks it quotes."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("n", [1023, 2047, 4095])
def test_algorithmic_bytes_per_grid_point(n):
    """Compulsory traffic of the three kernels of a step: the column convolution reads and
    writes the half spectrum (16 B per complex value) and reads the eigenvalues (8 B); the
    x-sweep reads the spectrum and u^n and writes X; the y-sweep reads X, u^n, u^{n-1},
    writes u^{n+1} and the next spectrum.  With N (M+1) spectrum values per grid that is
    40 + 32 + 48 = 120 B per grid point up to the (M+1)/N factor."""
    m = n + 1
    b = bench.algorithmic_bytes(n)
    spec = n * (m + 1) * 16
    assert b["cols_conv"] == 2 * spec + (m + 1) ** 2 * 8
    assert b["rows_rhs_gs"] == spec + 2 * n * n * 8
    assert b["cols_gs_fwd"] == spec + 4 * n * n * 8
    per_pt = sum(b[k] for k in bench.STEP_KERNELS) / (n * n)
    assert 120.0 <= per_pt < 120.0 * (1 + 4.0 / n)


def test_peaks():
    # 256 CUs x 4 SIMDs x 16 FP64 lanes x 2 (fma) x 2.4 GHz
    assert bench.FP64_VALU_PEAK_TFLOPS == pytest.approx(256 * 4 * 16 * 2 * 2.4e9 / 1e12, rel=2e-3)
    assert bench.HBM_PEAK_GBS == 8000.0
    assert bench.VALU_ISSUE_PEAK == pytest.approx(256 * 4 * 2.4e9 / 4)


def test_roofline_records_from_committed_profiles():
    """The traffic and ALU records are None or consistent with the algorithmic bytes (the
    measured traffic of the dominant kernel lies within 25% of its compulsory bytes)."""
    t = bench.traffic_record("cols_gs_fwd")
    if t is None:
        pytest.skip("counters taken on other kernel sources")
    alg = bench.algorithmic_bytes(4095)["cols_gs_fwd"]
    assert 0.95 * alg < t < 1.25 * alg
    v = bench.alu_view("cols_gs_fwd", 0.3)
    assert v is not None and v["bound"] == "alu" and 0.0 < v["frac"] < 1.0
