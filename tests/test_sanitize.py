"""The CPU test infrastructure under AddressSanitizer and
UndefinedBehaviorSanitizer: the oracle and the generator (driven by
tests/sanitize_driver.c over small instances, every rule and entry point,
and refused inputs) and the filter property check (tests/filter_check.cpp,
host build of the decoder's scoring header).  Host code only: nothing here
is built for or runs on the GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _have(tool):
    return shutil.which(tool) is not None


@pytest.mark.skipif(not _have("gcc"), reason="gcc not available")
def test_oracle_and_generator_under_sanitizers(tmp_path):
    exe = os.path.join(tmp_path, "sanitize_driver")
    subprocess.run(["gcc", "-std=c11", "-ffp-contract=off", *SAN,
                    os.path.join(ROOT, "tests", "sanitize_driver.c"),
                    os.path.join(ROOT, "oracle", "l0_oracle.c"),
                    os.path.join(ROOT, "gen", "l0gen.c"), "-o", exe, "-lm"], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("OK"), out.stdout
    assert "runtime error" not in out.stderr, out.stderr


@pytest.mark.skipif(not _have("g++"), reason="g++ not available")
def test_filter_check_under_sanitizers(tmp_path):
    exe = os.path.join(tmp_path, "filter_check_san")
    subprocess.run(["g++", "-std=c++17", "-ffp-contract=off", *SAN,
                    "-I" + os.path.join(ROOT, "paper_1508_01256_amd", "csrc"),
                    os.path.join(ROOT, "tests", "filter_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe, "2000"], capture_output=True, text=True, timeout=300, env=ENV)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("OK")
    assert "runtime error" not in out.stderr, out.stderr
