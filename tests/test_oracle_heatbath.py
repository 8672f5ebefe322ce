"""Oracle pins: the Kennedy-Pendleton SU(2) draw in multi-hit form and the
Cabibbo-Marinari SU(3) update with a frozen staple (Sec. 1, Sec. 2.1)."""
import numpy as np
import pytest

from exact_su3 import kp_acceptance, u_exact, x0_cdf, x0_mean
from paper_0904_0642_amd import workloads
from stats import jackknife_mean


@pytest.mark.parametrize("alpha", [0.7, 3.0, 12.5, 40.0])
def test_kp_single_hit_acceptance(oracle_mod, alpha):
    n = 30000
    acc = sum(oracle_mod.kp_draw(alpha, 1, 99, lid, 0, 0)[0] == 0 for lid in range(n))
    p = kp_acceptance(alpha)
    assert abs(acc / n - p) < 5 * np.sqrt(p * (1 - p) / n)


def test_kp_acceptance_matches_paper_ballpark():
    # Sec. 2.1 puts the single-hit acceptance near 97% at the couplings of interest; alpha = 2k/3
    # with k ~ 2(D-1) beta * <P> ~ 6 * 6 * 0.6 gives alpha ~ 14.
    assert 0.96 < kp_acceptance(14.0) < 0.98


@pytest.mark.parametrize("alpha", [0.7, 3.0, 12.5, 40.0])
def test_kp_x0_distribution(oracle_mod, alpha):
    n = 20000
    xs = []
    hits = []
    for lid in range(n):
        hit, x0, _ = oracle_mod.kp_draw(alpha, 200, 5, lid, 3, 1)
        assert hit >= 0
        xs.append(x0)
        hits.append(hit)
    xs = np.sort(np.array(xs))
    assert xs[0] >= -1.0 and xs[-1] <= 1.0
    m = x0_mean(alpha)
    var = np.var(xs)
    assert abs(xs.mean() - m) < 5 * np.sqrt(var / n)
    cdf = x0_cdf(alpha)(xs)
    emp = np.arange(1, n + 1) / n
    ks = max(np.max(emp - cdf), np.max(cdf - (emp - 1 / n)))
    assert ks < 1.95 / np.sqrt(n)           # 0.1% level of Kolmogorov's distribution
    # the accepted hit index is geometric with success probability p(alpha)
    p = kp_acceptance(alpha)
    assert abs(np.mean(np.array(hits) == 0) - p) < 5 * np.sqrt(p * (1 - p) / n)


def test_kp_multihit_gives_up_after_nhit(oracle_mod):
    # tiny alpha: acceptance ~ 1e-4 per hit, so 3 hits almost always fail and
    # exactly 3 proposals are counted
    fails = 0
    for lid in range(200):
        hit, _, att = oracle_mod.kp_draw(1e-3, 3, 1, lid, 0, 2)
        if hit < 0:
            fails += 1
            assert att == 3
        else:
            assert att == hit + 1
    assert fails > 190


@pytest.mark.parametrize("beff", [2.0, 8.0, 36.0])
def test_cm_frozen_staple(oracle_mod, beff):
    # Staple A = beff * V0 with V0 Haar: the CM chain samples
    # exp((beff/3) Re Tr(U V0)), so <(1/3) Re Tr(U V0)> = u(beff).
    # W = U A (not A U) matters here because V0 does not commute with U.
    rng = np.random.default_rng(int(beff * 10))
    v0 = workloads.random_su3(rng, 1)[0]
    a = beff * v0
    u = np.eye(3, dtype=complex)
    series = []
    for t in range(16000):
        u, _, _ = oracle_mod.cm_update_matrix(u, a, 8, 17, 5, t)
        if t >= 500:
            series.append(np.trace(u @ v0).real / 3)
    m, e = jackknife_mean(series, 32)
    assert abs(m - u_exact(beff)) < 5 * e + 1e-4


def test_cm_degenerate_staple_keeps_link(oracle_mod):
    rng = np.random.default_rng(1)
    u = workloads.random_su3(rng, 1)[0]
    un, at, ac = oracle_mod.cm_update_matrix(u, np.zeros((3, 3)), 8, 1, 0, 0)
    assert ac == [0, 0, 0] and at == [0, 0, 0]
    assert np.abs(un - u).max() < 1e-14


def test_cold_start_staple_and_plaquette(oracle_mod):
    # ordered start: every plaquette is 1 and every staple is 2(D-1) beta * 1
    for ext in ([4, 4, 4, 4], [4, 4], [2, 4, 2]):
        L = oracle_mod.Lattice(ext)
        L.cold_start()
        D = len(ext)
        p = L.plaquette(6.0)
        assert p[0] == 1.0 and p[2] == 1.0 and p[3] == 1.0
        assert p[5] == 6.0 * L.V * D * (D - 1) / 2
        for s in (0, 1, L.V - 1):
            for mu in range(D):
                assert np.array_equal(L.staple(0, s, mu, 6.0), 2 * (D - 1) * 6.0 * np.eye(3))


def test_link_margin_observes_without_changing(oracle_mod):
    # the threshold-margin probe (used to explain accept/reject flips between
    # platforms, Sec. 3) changes neither the links nor the sweep counter
    o = oracle_mod.Lattice([4, 4, 4, 4], seed=3)
    o.hot_start()
    o.sweep(5.8, nhit=8, nsweeps=2)
    before, sw = o.get_links(), o.sweep_counter
    m = o.link_margin(0, 5, 2, 5.8, nhit=8)
    assert np.array_equal(o.get_links(), before) and o.sweep_counter == sw
    assert 0.0 < m < 2.0
    # beta = 0: every projection is degenerate, no proposal is evaluated
    assert o.link_margin(0, 5, 2, 0.0, nhit=8) == float("inf")
    # ordered start, beta = 6, D = 4: subgroup (0,1) of the first link sees
    # W = 36 * 1, alpha = 24; the margin is at most that of its first
    # proposal, recomputed here from the Philox words of the counter
    # (link id, sweep 0, subgroup 0 hit 0 block 0, update stream)
    c = oracle_mod.Lattice([4, 4, 4, 4], seed=9)
    c.cold_start()
    s, mu = 0, 0
    words = oracle_mod.philox4x32_10([s * 4 + mu, 0, 0, 0], [9, 0])
    u = [oracle_mod.uniform(w) for w in words]
    delta = -(np.log(u[0]) + np.cos(2 * np.pi * u[1]) ** 2 * np.log(u[2])) / 24.0
    m0 = abs(u[3] ** 2 - (1.0 - 0.5 * delta))
    assert c.link_margin(0, s, mu, 6.0, nhit=1) <= m0 * (1 + 1e-12)
