"""The serving loop's admission arithmetic (paper_2002_05200_amd/csrc/
xd_admit.h) on the CPU: slot memory split inside the budget, cost classes,
and which queued requests a free slot admits.  The header holds no HIP code,
so tests/admit/admit_test.cpp builds with g++ here."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_admission_arithmetic(tmp_path):
    exe = str(tmp_path / "admit_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           f"-I{os.path.join(ROOT, 'include')}",
                           f"-I{os.path.join(ROOT, 'paper_2002_05200_amd', 'csrc')}",
                           os.path.join(ROOT, "tests", "admit", "admit_test.cpp"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ")
