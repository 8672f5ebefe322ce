"""Oracle pins: the Philox4x32-10 generator and the uniform map."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(t, 16) for t in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(oracle_mod):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert oracle_mod.philox4x32_10(ctr, key) == out


def test_uniform_map_endpoints(oracle_mod):
    # (r + 1) / 2^32 lies in (0, 1]: log(u) is always finite
    assert oracle_mod.uniform(0) == 2.0 ** -32
    assert oracle_mod.uniform(0xFFFFFFFF) == 1.0
    assert oracle_mod.uniform(0x7FFFFFFF) == 0.5


def test_uniform_moments(oracle_mod):
    u = []
    for i in range(5000):
        u += [oracle_mod.uniform(w) for w in oracle_mod.philox4x32_10([i, 7, 3, 0], [11, 13])]
    u = np.array(u)
    n = len(u)
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / n)
