"""The kernels' elementary functions of a Philox uniform u = (r+1)/2^32
(device_math.h: log_unit with its table, cos2_turn, sincos_turn), compiled for the host
from the same source and compared with mpmath at 200 bits: ln u to 1.5 ulp,
cos^2(2 pi u), sin and cos(2 pi u) to 2e-16 absolute in FP64 and 3e-7 in
FP32.  The words cover the ends of the range, the quarter-turn boundaries
of the reductions and random words."""
import os
import subprocess

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0904_0642_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "device_math_host.cpp")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("dm") / "device_math_host")
    r = subprocess.run(["hipcc", "-O2", "-std=c++17", "-I" + CSRC, "-I" + os.path.join(ROOT, "include"), SRC,
                        "-o", out], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def words():
    rng = np.random.default_rng(7)
    w = list(rng.integers(0, 2 ** 32, size=3000, dtype=np.uint64))
    w += [0, 1, 2, 3, 2 ** 32 - 1, 2 ** 32 - 2, 2 ** 31 - 1, 2 ** 31, 2 ** 31 + 1]
    # u near k/8 (t = 4u near k/2: the switch between quarter turns) and
    # near 2^-j (the binades of the logarithm's reduction), and m near sqrt(1/2)
    for k in range(1, 8):
        c = k * 2 ** 29 - 1
        w += [c - 1, c, c + 1]
    for j in range(1, 32):
        c = 2 ** (32 - j) - 1
        w += [c - 1, c, c + 1]
        # m near 3/4 (the switch of the logarithm's reduction) and near the
        # edges of its table bins
        s = int(round(2 ** 32 * 0.75 / 2 ** j)) - 1
        w += [s - 1, s, s + 1]
    for k in range(0, 128, 3):
        edge = (1 + k / 128) if k < 64 else (1 + k / 128) / 2
        s = int(round(2 ** 32 * edge / 2)) - 1
        w += [s - 1, s, s + 1]
    return [int(x) for x in w if 0 <= int(x) < 2 ** 32]


def test_elementary_functions_of_a_uniform(exe):
    ws = words()
    r = subprocess.run([exe], input="\n".join(map(str, ws)) + "\n", capture_output=True, text=True, check=True)
    rows = [[float.fromhex(v) for v in line.split()] for line in r.stdout.strip().splitlines()]
    assert len(rows) == len(ws)
    mp.mp.prec = 200
    worst = np.zeros(6)
    for w, (lg, c2, sd, cd, sf, cf) in zip(ws, rows):
        u = (mp.mpf(w) + 1) / 2 ** 32
        ln = mp.log(u)
        th = 2 * mp.pi * u
        s, c = mp.sin(th), mp.cos(th)
        ulp = np.spacing(abs(float(ln))) if ln != 0 else 2.0 ** -1074
        err = [abs(lg - ln) / ulp if ln != 0 else abs(lg), abs(c2 - c * c), abs(sd - s), abs(cd - c),
               abs(sf - s), abs(cf - c)]
        worst = np.maximum(worst, [float(e) for e in err])
    print("max errors: log %.2f ulp, cos^2 %.2e, sin/cos f64 %.2e %.2e, f32 %.2e %.2e" % tuple(worst))
    assert worst[0] <= 1.5
    assert worst[1] <= 2e-16 and worst[2] <= 2e-16 and worst[3] <= 2e-16
    assert worst[4] <= 3e-7 and worst[5] <= 3e-7


def test_log_table_matches_its_generator():
    # log_table.h is what gen_log_table.py writes (mpmath at 200 bits)
    import importlib.util
    import re
    spec = importlib.util.spec_from_file_location("gen_log_table", os.path.join(CSRC, "gen_log_table.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    want = gen.entries()
    text = open(os.path.join(CSRC, "log_table.h")).read()
    rows = re.findall(r"\{(\S+), (\S+), (\S+), 0\.0\}", text)
    assert len(rows) == 128
    got = [tuple(float.fromhex(v) for v in r) for r in rows]
    assert got == [tuple(w) for w in want]
    # the two bins next to m = 1 take c = 1 (r = m - 1 exactly, ln c = 0)
    assert got[0] == (1.0, 0.0, 0.0) and got[127] == (1.0, 0.0, 0.0)
