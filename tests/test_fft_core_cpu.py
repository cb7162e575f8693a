"""Host build of the FFT building blocks (no GPU): every transform length
L = 6 * 2^a up to 6144, forward and inverse, against a plain DFT in double."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_fft_core_matches_plain_dft(tmp_path):
    exe = tmp_path / "fft_core_check"
    src = os.path.join(ROOT, "tests", "fft_core_check.cpp")
    inc = os.path.join(ROOT, "paper_2509_19785_amd", "csrc")
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-I", inc, src, "-o", str(exe)], check=True,
                   capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout
    assert "all ok" in out.stdout
