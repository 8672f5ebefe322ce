"""The invariant-integer division of the FP32-12 kernel's site coordinates
(div_magic in layout.h), built for the host and checked against plain
integer division over every divisor up to 2^16 and larger ones (CPU)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0904_0642_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "div_magic_host.cpp")


def test_div_magic_matches_integer_division(tmp_path):
    exe = str(tmp_path / "div_magic_host")
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-I" + CSRC, SRC, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout
    assert out.stdout.strip().startswith("0 mismatches")
