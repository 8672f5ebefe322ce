"""Oracle pins: whole sweeps against exact results, the paper's statistics
and invariants of the checkerboard sweep."""
import json
import os

import numpy as np
import pytest

from exact_su3 import dlt_two_coupling_exact, u_exact
from stats import gaussian_difference_q, jackknife_mean

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _series(L, beta, nhit, ntherm, nmeas, beta1=None, col=0):
    L.sweep(beta, beta1, nhit=nhit, nsweeps=ntherm)
    out = []
    for _ in range(nmeas):
        L.sweep(beta, beta1, nhit=nhit, nsweeps=1)
        out.append(L.plaquette(beta, beta1)[col])
    return np.array(out)


@pytest.mark.parametrize("beta,nhit", [(4.0, 8), (4.0, 1), (1.0, 8)])
def test_2d_plaquette_exact(oracle_mod, beta, nhit):
    # In two dimensions <P> = u(beta) exactly up to O(u^{N_p}) (character
    # expansion on a closed surface); 16^2 torus.
    L = oracle_mod.Lattice([16, 16], seed=21, threads=4)
    L.hot_start()
    s = _series(L, beta, nhit, 200, 4000)
    m, e = jackknife_mean(s, 32)
    assert abs(m - u_exact(beta)) < 5 * e


@pytest.mark.parametrize("mask", [0b11, 0b01])
def test_2d_dlt_plaquette_exact(oracle_mod, mask):
    # A 2D double-layered torus (glued in both or in one direction) is again a
    # closed surface of genus one, so <P> = u(beta) as well.
    L = oracle_mod.Lattice([8, 8], nlat=2, dlt_mask=mask, seed=4, threads=2)
    L.hot_start()
    s = _series(L, 4.0, 8, 200, 4000)
    m, e = jackknife_mean(s, 32)
    assert abs(m - u_exact(4.0)) < 5 * e


def test_2d_dlt_two_couplings_exact(oracle_mod):
    # beta0 != beta1 on the 2D double-layered torus: per-layer averages and
    # the beta-weighted sum against the exact values (pins the tag rule)
    b0, b1 = 4.0, 2.0
    L = oracle_mod.Lattice([8, 8], nlat=2, dlt_mask=0b11, seed=6, threads=2)
    L.hot_start()
    L.sweep(b0, b1, nhit=8, nsweeps=200)
    rows = []
    for _ in range(4000):
        L.sweep(b0, b1, nhit=8, nsweeps=1)
        rows.append(L.plaquette(b0, b1)[[3, 4, 5]])
    rows = np.array(rows)
    exact = dlt_two_coupling_exact(8, 8, b0, b1)
    for k in range(3):
        m, e = jackknife_mean(rows[:, k], 32)
        assert abs(m - exact[k]) < 5 * e, (k, m, e, exact[k])


def test_4d_strong_coupling(oracle_mod):
    # Strong coupling: <P>_4D = u(beta) + O(u^5); at beta = 1, u^5 ~ 8e-7.
    L = oracle_mod.Lattice([6, 6, 6, 6], seed=8, threads=4)
    L.hot_start()
    s = _series(L, 1.0, 8, 50, 600)
    m, e = jackknife_mean(s, 20)
    assert abs(m - u_exact(1.0)) < 5 * e + 2e-6
    assert abs(u_exact(1.0) - (1 / 18 + 1 / 216)) < 2e-4


def test_table1_8x8x8x4(oracle_mod):
    # Table 1 (Sec. 3.3): periodic 8^3 4 at beta = 5.65, act = 0.538547(70)
    # (non-MPI row).  A short run here (errors ~1e-3) pins the beta and
    # action conventions (readings R-BETA, R-ACT).
    ref = GOLDEN["pbc_8x8x8x4_b5.65"]
    L = oracle_mod.Lattice(ref["extents"], seed=31, threads=8)
    L.cold_start()
    s = _series(L, ref["beta"], 1, 300, 1600)
    m, e = jackknife_mean(s, 16)
    m0, e0 = ref["actm"][0]
    assert gaussian_difference_q(m, e, m0, e0) > 1e-4
    assert abs(m - m0) < 0.006


def test_lat2test_reproduces_pbc(oracle_mod):
    # Sec. 3.4: with identical random numbers in both layers the DLT run
    # reproduces the PBC run; here link for link, bit for bit.
    ext = [4, 4, 2, 4]
    P = oracle_mod.Lattice(ext, seed=77)
    P.hot_start()
    T = oracle_mod.Lattice(ext, nlat=2, dlt_mask=0b1111, lat2test=True, seed=77)
    T.hot_start()
    for _ in range(3):
        P.sweep(5.65, nhit=2)
        T.sweep(5.65, nhit=2)
    a = P.get_links()
    b = T.get_links()
    assert np.array_equal(b[0], a[0]) and np.array_equal(b[1], a[0])
    pt, pp = T.plaquette(5.65), P.plaquette(5.65)
    assert np.allclose(pt[[0, 1, 2, 3, 4]], np.r_[pp[[0, 1, 2, 3]], pp[3]], rtol=1e-14, atol=0)


def test_slice_order_independence(oracle_mod):
    # Sites of one checkerboard slice are independent (Sec. 2): any site
    # order gives the same links, bit for bit.
    rng = np.random.default_rng(0)
    for ext, nlat, mask in (([4, 4, 4, 4], 1, 0), ([4, 2, 4, 2], 2, 0b1111)):
        A = oracle_mod.Lattice(ext, nlat=nlat, dlt_mask=mask, seed=3)
        A.hot_start()
        B = oracle_mod.Lattice(ext, nlat=nlat, dlt_mask=mask, seed=3)
        B.hot_start()
        for p in (0, 1):
            for mu in range(len(ext)):
                A.update_slice(p, mu, 5.8, 5.6, nhit=3)
                B.update_slice(p, mu, 5.8, 5.6, nhit=3, order=rng.permutation(B.V))
        assert np.array_equal(A.get_links(), B.get_links())


def test_resume_is_exact(oracle_mod):
    A = oracle_mod.Lattice([4, 4, 4, 2], seed=12)
    A.hot_start()
    A.sweep(5.7, nhit=8, nsweeps=5)
    B = oracle_mod.Lattice([4, 4, 4, 2], seed=12)
    B.hot_start()
    B.sweep(5.7, nhit=8, nsweeps=2)
    links, ctr = B.get_links(), B.sweep_counter
    C = oracle_mod.Lattice([4, 4, 4, 2], seed=12)
    C.set_links(links)
    C.sweep_counter = ctr
    C.sweep(5.7, nhit=8, nsweeps=3)
    assert ctr == 2 and C.sweep_counter == 5
    assert np.array_equal(A.get_links(), C.get_links())


def test_thread_count_invariance(oracle_mod):
    res = []
    for th in (1, 4):
        L = oracle_mod.Lattice([8, 8, 4, 4], seed=2, threads=th)
        L.hot_start()
        L.sweep(6.0, nhit=8, nsweeps=2)
        res.append(L.get_links())
    assert np.array_equal(res[0], res[1])


@pytest.mark.parametrize("ext,nlat,mask,b0,b1", [([4, 4, 4, 4], 1, 0, 6.0, 6.0),
                                                 ([4, 4, 2, 4], 2, 0b0111, 5.5, 6.5)])
def test_running_action_matches_recompute(oracle_mod, ext, nlat, mask, b0, b1):
    # Sec. 2.1/2.4: the action kept on record during updating must agree with
    # a direct recomputation.  Here: the beta-weighted trace sum.
    L = oracle_mod.Lattice(ext, nlat=nlat, dlt_mask=mask, seed=6)
    L.hot_start()
    t0 = L.plaquette(b0, b1)[5]
    st = L.sweep(b0, b1, nhit=8, nsweeps=6)
    t1 = L.plaquette(b0, b1)[5]
    assert abs(t0 + st["dtrace"] - t1) < 1e-11 * abs(t1) + 1e-9


def test_counters_and_acceptance(oracle_mod):
    L = oracle_mod.Lattice([4, 4, 4, 4], seed=1)
    L.cold_start()
    st = L.sweep(6.0, nhit=8, nsweeps=4)
    n_updates = 4 * 1024
    # every subgroup draws at least one proposal per link update, and with
    # n_hit = 8 at beta = 6 virtually every subgroup update is accepted
    assert np.all(st["attempts"] >= n_updates)
    assert np.all(st["accepts"] <= n_updates)
    assert np.all(st["accepts"] >= n_updates - 2)
    assert np.all(st["attempts"] < 1.1 * n_updates)
