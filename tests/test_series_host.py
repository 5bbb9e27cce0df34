"""Series for erfc and exp near zero (half-space moments) against the C
library: within 4 units of 2^-52 relative, compiled for the host from the
device header."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_erfc_and_exp_series_match_the_library(tmp_path):
    exe = str(tmp_path / 'series_check')
    subprocess.check_call(['g++', '-std=c++17', '-O1', '-D__HIP_PLATFORM_AMD__', '-I/opt/rocm/include',
                           '-I', os.path.join(ROOT, 'paper_2001_01570_amd', 'csrc'), '-I', os.path.join(ROOT, 'include'),
                           os.path.join(ROOT, 'tests', 'host', 'series_check.cpp'), '-o', exe],
                          stderr=subprocess.DEVNULL)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
