"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the library's host plan builder and the oracle, built with g++/gcc and the
sanitizers and run on clouds of several shapes, sizes and settings, including
the degenerate ones.  Any invalid access, leak or undefined operation fails
the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_plan_builder_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2202_04894_amd", "csrc")
    exe = str(tmp_path / "host_plan")
    _run(["g++", "-std=c++17", "-ffp-contract=off", "-pthread", *SAN, os.path.join(HERE, "host_plan_driver.cpp"),
          os.path.join(csrc, "plan_build.cpp"), os.path.join(csrc, "fourier_layout.cpp"), "-o", exe], tmp_path)
    out = _run([exe], tmp_path)
    assert "host plan driver: ok" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle")
    _run(["gcc", "-std=gnu11", "-ffp-contract=off", "-fopenmp", *SAN, os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "defmm_oracle.c"), "-o", exe, "-lm"], tmp_path)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe], cwd=tmp_path, capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "oracle driver: ok" in r.stdout
