"""Pins of the oracle's overrelaxation (reading R-OR: per SU(2) subgroup the
block k V of W = U A becomes k V^dag, so the local action is unchanged).

  * microcanonical: Re Tr(U A) is the same before and after, for general
    staples, to rounding; the link stays in SU(3) and does move;
  * whole lattices: an overrelaxation sweep keeps the action of every link at
    the moment it is updated, so the running trace change is rounding only;
  * statistics: heatbath sweeps interleaved with overrelaxation sweeps give
    the exact 2D plaquette u(beta) (overrelaxation alone is not ergodic, but
    it leaves the Boltzmann distribution invariant).
"""
import numpy as np
import pytest

from exact_su3 import u_exact
from paper_0904_0642_amd import workloads
from stats import gaussian_difference_q, jackknife_mean


def _rand_staple(rng, scale):
    # a general staple: a sum of six random SU(3) matrices times scale
    return scale * workloads.random_su3(rng, 6).sum(axis=0)


@pytest.mark.parametrize("scale", [0.3, 1.0, 6.0])
def test_reflection_keeps_the_local_action(oracle_mod, scale):
    rng = np.random.default_rng(3)
    moved = []
    for _ in range(200):
        u = workloads.random_su3(rng, 1)[0]
        a = _rand_staple(rng, scale)
        v = oracle_mod.reflect_matrix(u, a)
        before, after = np.trace(u @ a).real, np.trace(v @ a).real
        assert abs(after - before) <= 1e-12 * max(1.0, abs(before))
        assert np.abs(v @ v.conj().T - np.eye(3)).max() < 1e-13
        assert abs(np.linalg.det(v) - 1.0) < 1e-13
        moved.append(np.abs(v - u).max())
    assert np.median(moved) > 0.05


def test_reflection_of_a_zero_staple_is_the_identity_map(oracle_mod):
    rng = np.random.default_rng(4)
    u = workloads.random_su3(rng, 1)[0]
    v = oracle_mod.reflect_matrix(u, np.zeros((3, 3), dtype=complex))
    assert np.abs(v - u).max() < 1e-14


@pytest.mark.parametrize("ext,nlat,mask,b0,b1", [((4, 4, 4, 4), 1, 0, 6.0, 6.0), ((4, 6, 2, 4), 2, 0b1111, 5.5, 6.5)])
def test_overrelaxation_sweep_keeps_the_action(oracle_mod, ext, nlat, mask, b0, b1):
    L = oracle_mod.Lattice(list(ext), nlat=nlat, dlt_mask=mask, seed=5)
    L.hot_start()
    L.sweep(b0, b1, nhit=4, nsweeps=3)
    t0 = L.plaquette(b0, b1)[5]
    sw0 = L.sweep_counter
    st = L.overrelax(b0, b1, nsweeps=2)
    t1 = L.plaquette(b0, b1)[5]
    n = 2 * nlat * int(np.prod(ext)) * len(ext)
    assert list(st["attempts"]) == [n] * 3 and list(st["accepts"]) == [n] * 3
    assert abs(st["dtrace"]) < 1e-9 * abs(t0)
    assert abs(t1 - t0) < 1e-9 * abs(t0)
    assert L.sweep_counter == sw0 + 2


def test_mixed_sweeps_give_the_exact_2d_plaquette(oracle_mod):
    L = oracle_mod.Lattice([16, 16], seed=8)
    L.hot_start()
    beta = 4.0
    for _ in range(50):
        L.sweep(beta, nhit=8, nsweeps=1)
        L.overrelax(beta, nsweeps=2)
    series = []
    for _ in range(3000):
        L.sweep(beta, nhit=8, nsweeps=1)
        L.overrelax(beta, nsweeps=2)
        series.append(L.plaquette(beta)[0])
    m, e = jackknife_mean(np.array(series), 32)
    q = gaussian_difference_q(m, e, u_exact(beta), 0.0)
    print(f"16^2 beta=4 HB+2OR: {m:.6f}({e * 1e6:.0f}) exact {u_exact(beta):.6f} Q={q:.2f}")
    assert q > 1e-3
