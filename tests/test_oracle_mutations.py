"""The pins catch planted mistakes.

Each case copies oracle/su3_oracle.c, plants one plausible mistake (a
dropped term, a wrong sign, a transposed or un-daggered operand, a wrong
index, constant or acceptance test), builds the copy with the same compiler
flags and runs the oracle's CPU pins against it in a subprocess
(SU3HB_ORACLE_LIB points the oracle package at the copy).  A mistake counts
as caught when at least one pin fails.  Nothing here touches a GPU or the
GPU library.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "su3_oracle.c")

# name: (text in the oracle, planted replacement)
MUTANTS = {
    "philox multiplier": ("(uint64_t)0xD2511F53u * (uint64_t)c0", "(uint64_t)0xD2511F57u * (uint64_t)c0"),
    "philox nine rounds": ("round < 10", "round < 9"),
    "uniform map reaches 0": ("((double)r + 1.0) * 0x1p-32", "((double)r) * 0x1p-32"),
    "backward staple dropped": ("A->m[i][j] += bf * f.m[i][j] + bb * bk.m[i][j];", "A->m[i][j] += bf * f.m[i][j];"),
    "forward staple without dagger": ("su3 b = mat_adj(link_at(L, l_xpnu, s_xpnu, mu));",
                                      "su3 b = *link_at(L, l_xpnu, s_xpnu, mu);"),
    "backward staple wrong site": ("neighbor(L, l_xpmu, s_xpmu, nu, -1, &l_xpmu_mnu, &s_xpmu_mnu);",
                                   "neighbor(L, layer, s, nu, -1, &l_xpmu_mnu, &s_xpmu_mnu);"),
    "projection sign of a1": ("double a1 = cimag(w.m[i][j] + w.m[j][i]) / 2;",
                              "double a1 = cimag(w.m[i][j] - w.m[j][i]) / 2;"),
    "W = A U instead of U A": ("su3 w = mat_mul(u, a);", "su3 w = mat_mul(a, u);"),
    "alpha = k/3 (beta = 2/g^2)": ("double alpha = 2.0 * k / 3.0;", "double alpha = k / 3.0;"),
    "KP without cos^2": ("double delta = -(log(r[0]) + c * c * log(r[2])) / alpha;",
                         "double delta = -(log(r[0]) + log(r[2])) / alpha;"),
    "KP acceptance R4 not R4^2": ("if (r[3] * r[3] <= 1.0 - 0.5 * delta) {", "if (r[3] <= 1.0 - 0.5 * delta) {"),
    "sphere direction cos(theta) = R5": ("double cth = 2.0 * r[0] - 1.0;", "double cth = r[0];"),
    "third row not conjugated": ("u->m[2][0] = conj(a[1] * b[2] - a[2] * b[1]);",
                                 "u->m[2][0] = (a[1] * b[2] - a[2] * b[1]);"),
    "Gram-Schmidt projection dropped": ("for (int c = 0; c < 3; ++c) u->m[1][c] -= d * u->m[0][c];", ""),
    "no layer flip on a glued wrap": ("*lo = (wrapped && L->nlat == 2 && ((L->dlt_mask >> dir) & 1u)) ? 1 - layer : layer;",
                                      "*lo = layer;"),
    "forward staple ignores the tag rule": ("double bf = tags == 0 ? beta0 : beta1;", "double bf = beta0;"),
    "timelike planes mislabelled": ("if (nu == D - 1) time += P; else space += P;",
                                    "if (mu == 0) time += P; else space += P;"),
    "overrelaxation r = V^dag instead of V^dag V^dag": ("R[p][q] = Vd[p][0] * Vd[0][q] + Vd[p][1] * Vd[1][q];",
                                                         "R[p][q] = Vd[p][q];"),
    "lat2test keeps the layer in the link id": ("long base = L->lat2test ? 0 : (long)layer * L->V;",
                                                "long base = (long)layer * L->V;"),
}

PINS = ["tests/test_oracle_rng.py", "tests/test_oracle_geometry.py", "tests/test_oracle_su3.py",
        "tests/test_oracle_heatbath.py", "tests/test_oracle_overrelax.py", "tests/test_oracle_physics.py"]


@pytest.fixture(scope="module")
def source():
    return open(SRC).read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(source, name):
    old, new = MUTANTS[name]
    # the mistake goes in wherever the line occurs (the heatbath and the
    # overrelaxation share the subgroup projection)
    assert source.count(old) >= 1, f"mutation site for '{name}' not found in the oracle"
    with tempfile.TemporaryDirectory() as tmp:
        src = os.path.join(tmp, "su3_oracle.c")
        lib = os.path.join(tmp, "liboracle.so")
        open(src, "w").write(source.replace(old, new))
        subprocess.run(["gcc", "-std=gnu11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                        "-w", src, "-lm", "-o", lib], check=True)
        env = dict(os.environ, SU3HB_ORACLE_LIB=lib, OMP_NUM_THREADS="4")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                            "--deselect", "tests/test_oracle_physics.py::test_table1_8x8x8x4"] + PINS,
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr).strip().splitlines()[-3:]
    print(f"{name}: exit {r.returncode}: {' | '.join(tail)}")
    # exit status 1: a pin failed (0 would mean every pin passed with the mistake in place)
    assert r.returncode == 1, f"no pin caught '{name}': {tail}"
