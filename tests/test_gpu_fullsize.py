"""Parity at the benchmark sizes, in the launch configuration the benchmark
uses (autotuned), on sampled links.

After one GPU sweep the state before slice (p, mu) is known exactly: links
of the slices already done come from the GPU's result, all others from the
start.  The oracle rebuilds that state and recomputes sampled links of every
slice one by one.  Properties that hold at any size (unitarity, the running
action against a recomputation) are checked on the whole lattice.
"""
import sys

import numpy as np
import pytest

import paper_0904_0642_amd as su3hb

pytestmark = pytest.mark.gpu

NSAMPLE = 48


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    su3hb.lib()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def parities(ext):
    idx = np.arange(int(np.prod(ext)), dtype=np.int64)
    par = np.zeros_like(idx)
    stride = 1
    for n in ext:
        par += (idx // stride) % n
        stride *= n
    return (par & 1).astype(np.int8)


def sampled_sweep_parity(oracle_mod, ext, prec, beta, slices, tol, nlat=1, mask=0):
    say(f"case full size ext={ext} nlat={nlat} mask={mask:b} prec={prec} beta={beta}")
    g = su3hb.Lattice(ext, nlat=nlat, dlt_mask=mask, precision=prec, seed=1)
    g.autotune(400)
    say(f"  launch {g.get_launch()}")
    L0 = g.get_links()
    t0 = g.plaquette(beta)[5]
    st = g.sweep(beta, n_hit=8, n_sweeps=1, stats=True)
    L1 = g.get_links()
    t1 = g.plaquette(beta)[5]
    # the running action kept during the sweep equals a recomputation
    say(f"  running trace {t0 + st['dtrace']:.10f} recomputed {t1:.10f}")
    rel = abs(t0 + st["dtrace"] - t1) / abs(t1)
    fp64 = prec in (su3hb.FP64_18, su3hb.FP64_12)
    assert rel < (1e-11 if fp64 else 1e-5)
    # every link still in SU(3)
    u = L1.reshape(-1, 3, 3)
    for c0 in range(0, u.shape[0], 1 << 22):
        blk = u[c0:c0 + (1 << 22)]
        d = np.abs(np.einsum("nij,nkj->nik", blk, blk.conj()) - np.eye(3)).max()
        assert d < (1e-12 if fp64 else 1e-6)
    del u

    par = parities(ext)
    D = len(ext)
    rng = np.random.default_rng(2024)
    o = oracle_mod.Lattice(list(ext), nlat=nlat, dlt_mask=mask, seed=1, threads=16)
    state = L0.copy()
    order = [(p, mu) for p in (0, 1) for mu in range(D)]
    worst = 0.0
    for k, (p, mu) in enumerate(order):
        if (p, mu) in slices:
            o.set_links(state)
            o.sweep_counter = 0
            sites = rng.choice(np.flatnonzero(par == p), size=NSAMPLE, replace=False)
            layers = rng.integers(0, nlat, size=NSAMPLE)
            for s, lay in zip(sites, layers):
                o.update_link(int(lay), int(s), mu, beta, beta, 8)
                d = float(np.abs(o.get_link(int(lay), int(s), mu) - L1[lay, s, mu]).max())
                worst = max(worst, d)
            say(f"  slice (p={p}, mu={mu}): {NSAMPLE} sampled links, max |dU| so far {worst:.3e}")
        # the slice is done: its links take the GPU's values
        mask_p = par == p
        state[:, mask_p, mu] = L1[:, mask_p, mu]
    assert worst <= tol
    g.close()


ALL_SLICES = {(p, mu) for p in (0, 1) for mu in range(4)}


@pytest.mark.timeout(300)
def test_48x48x48x48_fp64(oracle_mod):
    ext = (48, 48, 48, 48)
    sampled_sweep_parity(oracle_mod, ext, su3hb.FP64_18, 6.2, ALL_SLICES, 1e-10)


@pytest.mark.timeout(600)
def test_64x64x64x64_fp32_12(oracle_mod):
    ext = (64, 64, 64, 64)
    sampled_sweep_parity(oracle_mod, ext, su3hb.FP32_12, 6.2, ALL_SLICES, 1e-4)


@pytest.mark.timeout(300)
def test_48x48x48x48_fp64_12(oracle_mod):
    # the benchmark's full-size FP64-12 leg: two stored rows, row 2 rebuilt
    # on every load, against the oracle's full matrices
    ext = (48, 48, 48, 48)
    sampled_sweep_parity(oracle_mod, ext, su3hb.FP64_12, 6.2, ALL_SLICES, 1e-10)


@pytest.mark.timeout(600)
def test_64x64x64x64_fp32_18_past_4gb(oracle_mod):
    # 4.83 GB of links: the slab of U_3 on odd sites starts 4.23 GB into the
    # buffer, so slice (1, 3) updates links whose byte offsets need more than
    # 32 bits, and slice (0, 3) reads them as its U_mu neighbours
    ext = (64, 64, 64, 64)
    sampled_sweep_parity(oracle_mod, ext, su3hb.FP32_18, 6.2, {(0, 3), (1, 3)}, 1e-4)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec,tol", [(su3hb.FP64_18, 1e-10), (su3hb.FP32_18, 1e-4), (su3hb.FP32_12, 1e-4)])
def test_double_layered_2x24x24x24x8(oracle_mod, prec, tol):
    # the double-layered torus of two 24^3 x 8 layers glued in every
    # direction at beta = 5.69, in the launch shape the benchmark uses:
    # sampled links of both layers in all eight slices of one sweep
    sampled_sweep_parity(oracle_mod, (24, 24, 24, 8), prec, 5.69, ALL_SLICES, tol, nlat=2, mask=0b1111)
