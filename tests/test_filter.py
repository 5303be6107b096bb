"""CPU property check of the decoder's column scoring (host build of
csrc/l0_filter.h with g++): the bit-sliced counts, the bucket-word filter's
definition, exact_score against the l0-decrease of eq. (selection_l0), and
that the filter never rejects a column the exact score selects."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_filter_properties(tmp_path):
    exe = os.path.join(tmp_path, "filter_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off",
                    "-I" + os.path.join(ROOT, "paper_1508_01256_amd", "csrc"),
                    os.path.join(ROOT, "tests", "filter_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe, "20000"], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("OK")
