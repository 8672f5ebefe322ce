"""GPU <-> oracle parity through the C ABI.

Both sides draw the same Philox random numbers, so after one sweep from a
shared start every link must agree to rounding:
  * FP64 storage: max |U_gpu - U_oracle| <= 1e-10 per matrix element
    (the bound the build targets; libm vs device log/cos/sqrt differ by ulps);
  * FP32 storage: <= 1e-4 (FP32 staple products; the error is printed).
Cases span several blocks with ragged tails, D = 2..6, the double-layered
torus (beta0 != beta1), lat2test, and the edge cases of the interface.
"""
import sys

import numpy as np
import pytest

import paper_0904_0642_amd as su3hb
from paper_0904_0642_amd import workloads

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    su3hb.lib()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pair(oracle_mod, ext, nlat=1, mask=0, lat2test=False, prec=su3hb.FP64_18, start=su3hb.HOT, seed=1,
         threads=8):
    say(f"case ext={ext} nlat={nlat} mask={mask} lat2test={lat2test} prec={prec} start={start} seed={seed}")
    g = su3hb.Lattice(ext, nlat=nlat, dlt_mask=mask, lat2test=lat2test, precision=prec, start=start, seed=seed)
    o = oracle_mod.Lattice(ext, nlat=nlat, dlt_mask=mask, lat2test=lat2test, seed=seed, threads=threads)
    if start == su3hb.COLD:
        o.cold_start()
    else:
        o.hot_start()
    return g, o


def maxdiff(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max())


# ---------------------------------------------------------------------------

def test_config1_cold_4x4x4x4(oracle_mod):
    # 4^4, beta = 6.0, ordered start, n_hit = 8, seed 1, 20 sweeps, FP64
    g, o = pair(oracle_mod, [4, 4, 4, 4], start=su3hb.COLD, seed=1)
    assert maxdiff(g.get_links(), o.get_links()) == 0.0
    st_g = g.sweep(6.0, n_hit=8, n_sweeps=1, stats=True)
    st_o = o.sweep(6.0, nhit=8, nsweeps=1)
    d = maxdiff(g.get_links(), o.get_links())
    say(f"  after 1 sweep: max |dU| = {d:.3e}")
    assert d <= TOL64
    assert list(st_g["attempts"]) == list(st_o["attempts"])
    assert list(st_g["accepts"]) == list(st_o["accepts"])
    assert st_g["link_updates"] == 1024
    assert abs(st_g["dtrace"] - st_o["dtrace"]) < 1e-9
    # per-sweep plaquette over the remaining 19 sweeps
    series = g.sweep_measure(6.0, n_hit=8, n_sweeps=19)
    ref = []
    for _ in range(19):
        o.sweep(6.0, nhit=8, nsweeps=1)
        ref.append(o.plaquette(6.0))
    ref = np.array(ref)
    dp = np.abs(series[:, :4] - ref[:, :4]).max(axis=1)
    say(f"  per-sweep |d<P>| max over 19 sweeps = {dp.max():.3e}; first = {dp[0]:.3e}")
    assert dp.max() < 1e-8
    assert g.get_state() == (1, 20)


@pytest.mark.parametrize("ext,seed", [([4, 4, 4, 4], 1), ([6, 4, 2, 10], 3), ([16, 16, 16, 16], 1)])
def test_hot_start_matches(oracle_mod, ext, seed):
    g, o = pair(oracle_mod, ext, seed=seed)
    d = maxdiff(g.get_links(), o.get_links())
    say(f"  hot start max |dU| = {d:.3e}")
    assert d <= 1e-12


@pytest.mark.parametrize("beta", [5.7, 6.0])
def test_16x16x16x16_one_sweep(oracle_mod, beta):
    g, o = pair(oracle_mod, [16, 16, 16, 16], seed=1, threads=16)
    g.sweep(beta, n_hit=8, n_sweeps=1)
    o.sweep(beta, nhit=8, nsweeps=1)
    d = maxdiff(g.get_links(), o.get_links())
    say(f"  16^4 beta={beta}: max |dU| = {d:.3e}")
    assert d <= TOL64
    pg = g.plaquette(beta)
    po = o.plaquette(beta)
    assert np.allclose(pg[[0, 1, 2, 3, 5]], po[[0, 1, 2, 3, 5]], rtol=1e-12, atol=0)


@pytest.mark.parametrize("ext", [[32, 32], [4, 6], [6, 4, 8], [4, 4, 2, 4, 2], [2, 4, 2, 2, 2, 4],
                                 [2, 2, 2, 2], [10, 2, 6, 4]])
def test_dimensions_and_ragged(oracle_mod, ext):
    g, o = pair(oracle_mod, ext, seed=5)
    for _ in range(2):
        g.sweep(5.8, n_hit=4, n_sweeps=1)
        o.sweep(5.8, nhit=4, nsweeps=1)
    d = maxdiff(g.get_links(), o.get_links())
    say(f"  {ext}: max |dU| after 2 sweeps = {d:.3e}")
    assert d <= TOL64
    pg, po = g.plaquette(5.8), o.plaquette(5.8)
    good = ~np.isnan(po)
    assert np.array_equal(np.isnan(pg), np.isnan(po))
    assert np.allclose(pg[good], po[good], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("mask,b0,b1", [(0b1111, 5.5, 6.0), (0b0111, 5.65, 5.9), (0b0000, 5.6, 6.1),
                                        (0b1000, 6.0, 6.0)])
def test_double_layered_torus(oracle_mod, mask, b0, b1):
    g, o = pair(oracle_mod, [4, 6, 4, 2], nlat=2, mask=mask, seed=9)
    st_g = g.sweep(b0, b1, n_hit=8, n_sweeps=2, stats=True)
    st_o = o.sweep(b0, b1, nhit=8, nsweeps=2)
    d = maxdiff(g.get_links(), o.get_links())
    say(f"  DLT mask={mask:04b} beta=({b0},{b1}): max |dU| = {d:.3e}")
    assert d <= TOL64
    assert abs(st_g["dtrace"] - st_o["dtrace"]) < 1e-9 * max(1.0, abs(st_o["dtrace"]))
    pg, po = g.plaquette(b0, b1), o.plaquette(b0, b1)
    assert np.allclose(pg, po, rtol=1e-12, atol=0, equal_nan=True)


def test_lat2test_layers_equal_torus(oracle_mod):
    ext = [4, 4, 2, 4]
    t = su3hb.Lattice(ext, nlat=2, dlt_mask=0b1111, lat2test=True, seed=44)
    p = su3hb.Lattice(ext, seed=44)
    t.sweep(5.65, n_hit=8, n_sweeps=3)
    p.sweep(5.65, n_hit=8, n_sweeps=3)
    lt, lp = t.get_links(), p.get_links()
    # the two layers draw the same numbers: identical to each other bit for
    # bit; the torus scales its staple once instead of per plaquette, so it
    # agrees to rounding
    assert np.array_equal(lt[0], lt[1])
    assert maxdiff(lt[0], lp[0]) <= 1e-12


@pytest.mark.parametrize("prec", [su3hb.FP32_18, su3hb.FP32_12])
@pytest.mark.parametrize("ext", [[8, 8, 8, 4], [6, 4, 2, 10]])
def test_fp32_storage_one_sweep(oracle_mod, prec, ext):
    # shared start: the oracle takes the FP32-rounded links the GPU holds;
    # 6x4x2x10 has 240 links per slab, so its last tile of 64 is partial
    g, o = pair(oracle_mod, ext, prec=prec, seed=2)
    start = g.get_links()
    o.set_links(start)
    g.sweep(6.0, n_hit=8, n_sweeps=1)
    o.sweep(6.0, nhit=8, nsweeps=1)
    d = maxdiff(g.get_links(), o.get_links())
    say(f"  prec={prec}: max |dU| after 1 sweep = {d:.3e}")
    assert d <= TOL32
    # links stay in SU(3) to FP32 rounding
    u = g.get_links().reshape(-1, 3, 3)
    unit = np.abs(np.einsum("nij,nkj->nik", u, u.conj()) - np.eye(3)).max()
    assert unit < 1e-6


@pytest.mark.parametrize("ext", [[8, 8, 8, 4], [6, 4, 2, 10], [16, 8]])
def test_fp64_12_storage_matches_oracle(oracle_mod, ext):
    # 12-real FP64 storage rebuilds row 2 = conj(row0 x row1) on load: the same
    # SU(3) matrix to rounding, so the FP64 bound holds
    g, o = pair(oracle_mod, ext, prec=su3hb.FP64_12, seed=23)
    assert maxdiff(g.get_links(), o.get_links()) <= 1e-12
    for _ in range(2):
        g.sweep(5.8, n_hit=8, n_sweeps=1)
        o.sweep(5.8, nhit=8, nsweeps=1)
    d = maxdiff(g.get_links(), o.get_links())
    say(f"  fp64-12 {ext}: max |dU| after 2 sweeps = {d:.3e}")
    assert d <= TOL64
    pg, po = g.plaquette(5.8), o.plaquette(5.8)
    assert np.allclose(pg, po, rtol=1e-12, atol=0, equal_nan=True)


def test_plaquette_of_same_links(oracle_mod):
    g, o = pair(oracle_mod, [8, 4, 6, 4], seed=13)
    o.sweep(5.9, nhit=2, nsweeps=1)
    g.set_links(o.get_links())
    assert np.allclose(g.plaquette(5.9), o.plaquette(5.9), rtol=1e-13, atol=0, equal_nan=True)


def test_set_links_rejects_non_su3(oracle_mod):
    g = su3hb.Lattice([4, 4, 2, 2], seed=3)
    good = g.get_links()
    bad = good.copy()
    bad[0, 5, 1] *= 1.001
    with pytest.raises(su3hb.SU3HBError) as ei:
        g.set_links(bad)
    assert ei.value.code == su3hb.ENOTSU3
    nan = good.copy()
    nan[0, 7, 0, 1, 1] = np.nan
    with pytest.raises(su3hb.SU3HBError):
        g.set_links(nan)
    assert np.array_equal(g.get_links(), good)            # unchanged after a failed set
    with pytest.raises(su3hb.SU3HBError):
        su3hb.su3hb_set_links(g.handle, good.view(np.float64).reshape(-1)[:-18])
    g.set_links(good)
    assert np.array_equal(g.get_links(), good)


def test_sweep_argument_errors():
    g = su3hb.Lattice([4, 4, 2, 2], seed=3)
    for bad in (dict(n_hit=0), dict(n_hit=40000), dict(n_sweeps=-1)):
        kw = dict(n_hit=8, n_sweeps=1)
        kw.update(bad)
        with pytest.raises(su3hb.SU3HBError) as ei:
            g.sweep(6.0, **kw)
        assert ei.value.code == su3hb.EINVAL
    with pytest.raises(su3hb.SU3HBError):
        g.sweep(float("nan"))
    g.sweep(6.0, n_sweeps=0)
    assert g.get_state()[1] == 0
    # the Philox sweep index is 32 bits: no state past it, no sweep across it
    with pytest.raises(su3hb.SU3HBError) as ei:
        g.set_state(3, 2 ** 32)
    assert ei.value.code == su3hb.EINVAL
    g.set_state(3, 2 ** 32 - 1)
    with pytest.raises(su3hb.SU3HBError) as ei:
        g.sweep(6.0, n_sweeps=2)
    assert ei.value.code == su3hb.EINVAL
    with pytest.raises(su3hb.SU3HBError):
        g.overrelax(6.0, n_sweeps=2)
    g.sweep(6.0, n_sweeps=1)
    assert g.get_state() == (3, 2 ** 32)


def test_zero_beta_is_degenerate(oracle_mod):
    # beta = 0: every staple is zero, so every SU(2) projection is degenerate
    # and every hit is rejected (no proposal is even counted); from the
    # ordered start the links stay exactly 1, from a random start they only
    # pass through reunitarisation
    g, o = pair(oracle_mod, [4, 4, 2, 6], start=su3hb.COLD, seed=4)
    st = g.sweep(0.0, n_hit=8, n_sweeps=2, stats=True)
    eye = np.broadcast_to(np.eye(3), g.get_links().shape)
    assert np.array_equal(g.get_links(), eye)
    assert list(st["attempts"]) == [0, 0, 0] and list(st["accepts"]) == [0, 0, 0]
    g, o = pair(oracle_mod, [4, 4, 2, 6], seed=4)
    st = g.sweep(0.0, n_hit=8, n_sweeps=1, stats=True)
    st_o = o.sweep(0.0, nhit=8, nsweeps=1)
    assert list(st["attempts"]) == [0, 0, 0] and list(st_o["attempts"]) == [0, 0, 0]
    assert maxdiff(g.get_links(), o.get_links()) <= 1e-13


@pytest.mark.parametrize("beta,n_hit", [(5.7, 1), (-2.0, 8), (0.3, 200)])
def test_hit_counts_and_signs(oracle_mod, beta, n_hit):
    # the paper's default single hit, a negative coupling (the projection
    # norm absorbs the sign), and a weak coupling with many rejections that
    # reaches deep into the hit counter
    g, o = pair(oracle_mod, [6, 4, 4, 4], seed=6)
    st_g = g.sweep(beta, n_hit=n_hit, n_sweeps=1, stats=True)
    st_o = o.sweep(beta, nhit=n_hit, nsweeps=1)
    d = maxdiff(g.get_links(), o.get_links())
    say(f"  beta={beta} n_hit={n_hit}: max |dU| = {d:.3e}, attempts {list(st_g['attempts'])}")
    assert d <= TOL64
    assert list(st_g["attempts"]) == list(st_o["attempts"])
    assert list(st_g["accepts"]) == list(st_o["accepts"])


@pytest.mark.parametrize("ext,nlat,mask,b0,b1,prec,tol", [
    ([8, 4, 4, 6], 1, 0, 6.0, 6.0, su3hb.FP64_18, TOL64),
    ([4, 6, 4, 2], 2, 0b1111, 5.5, 6.2, su3hb.FP64_18, TOL64),
    ([6, 4, 8], 1, 0, 5.0, 5.0, su3hb.FP64_12, TOL64),
    ([8, 4, 4, 6], 1, 0, 6.0, 6.0, su3hb.FP32_12, TOL32)])
def test_overrelaxation_matches_oracle(oracle_mod, ext, nlat, mask, b0, b1, prec, tol):
    # one heatbath sweep, then overrelaxation sweeps (no random numbers):
    # two in FP64 storage, one in FP32 storage (the FP32 bar is one update
    # per link from a shared start); counters are the reflections, the action
    # change is rounding only
    n_or = 2 if prec in (su3hb.FP64_18, su3hb.FP64_12) else 1
    g, o = pair(oracle_mod, ext, nlat=nlat, mask=mask, prec=prec, seed=12)
    if prec != su3hb.FP64_18:
        o.set_links(g.get_links())
    g.sweep(b0, b1, n_hit=8, n_sweeps=1)
    o.sweep(b0, b1, nhit=8, nsweeps=1)
    if prec in (su3hb.FP32_18, su3hb.FP32_12):
        o.set_links(g.get_links())
    t0 = g.plaquette(b0, b1)[5]
    st_g = g.overrelax(b0, b1, n_sweeps=n_or, stats=True)
    st_o = o.overrelax(b0, b1, nsweeps=n_or)
    d = maxdiff(g.get_links(), o.get_links())
    say(f"  OR ext={ext} nlat={nlat} prec={prec}: max |dU| = {d:.3e}, dtrace {st_g['dtrace']:.2e}")
    assert d <= tol
    assert list(st_g["attempts"]) == list(st_o["attempts"]) == [n_or * nlat * int(np.prod(ext)) * len(ext)] * 3
    rel = 1e-11 if prec in (su3hb.FP64_18, su3hb.FP64_12) else 1e-5
    assert abs(st_g["dtrace"]) <= rel * abs(t0)
    assert abs(g.plaquette(b0, b1)[5] - t0) <= rel * abs(t0)
    assert g.get_state()[1] == o.sweep_counter == 1 + n_or


def test_overrelaxation_graphs_equal_direct_launches():
    # heatbath and overrelaxation calls alternating through the graph cache
    # give the same links as the same sweeps launched kernel by kernel
    a = su3hb.Lattice([8, 8, 4, 4], seed=31)
    b = su3hb.Lattice([8, 8, 4, 4], seed=31)
    for _ in range(3):
        a.sweep(5.9, n_hit=8, n_sweeps=1)
        a.overrelax(5.9, n_sweeps=2)
        b.sweep_timed(5.9, n_hit=8, n_sweeps=1)
        b.sweep_timed(5.9, n_hit=0, n_sweeps=2)
    assert np.array_equal(a.get_links(), b.get_links(), equal_nan=True)
    assert a.get_state() == b.get_state()


@pytest.mark.parametrize("ext,mask,b0,b1,prec,tol", [
    ([4, 6, 4, 2], 0b1111, 5.5, 6.2, su3hb.FP64_18, 1e-13),
    ([8, 8, 4, 4], 0b0111, 5.9, 5.9, su3hb.FP64_18, 1e-13),
    ([6, 4, 8], 0b101, 5.0, 6.5, su3hb.FP64_12, 1e-13),
    ([16, 8], 0b11, 4.0, 2.0, su3hb.FP64_18, 1e-13),
    ([8, 8, 8, 4], 0b1111, 5.55, 5.55, su3hb.FP32_18, 2e-6),
    ([8, 8, 4, 4], 0b1000, 5.6, 6.0, su3hb.FP32_12, 2e-6)])
def test_fused_measurement_two_layers(ext, mask, b0, b1, prec, tol):
    # two layers: the parity-1 slices sort the plaquette terms into three
    # classes (base layer, tag sum); totals, spacelike/timelike, per layer and
    # the beta-weighted sum equal the standalone kernel on the same links
    a = su3hb.Lattice(ext, nlat=2, dlt_mask=mask, seed=23, precision=prec)
    b = su3hb.Lattice(ext, nlat=2, dlt_mask=mask, seed=23, precision=prec)
    fused = a.sweep_measure(b0, b1, n_hit=8, n_sweeps=4)
    sep = []
    for _ in range(4):
        b.sweep(b0, b1, n_hit=8, n_sweeps=1)
        sep.append(b.plaquette(b0, b1))
    sep = np.array(sep)
    assert np.array_equal(a.get_links(), b.get_links())
    assert np.array_equal(np.isnan(fused), np.isnan(sep))
    good = ~np.isnan(sep)
    d = np.abs(fused[good] - sep[good]) / np.maximum(1.0, np.abs(sep[good]))
    say(f"  two layers ext={ext} mask={mask:b} beta=({b0},{b1}) prec={prec}: max rel diff = {d.max():.3e}")
    assert d.max() <= tol


def test_fp64_12_chain_equals_fp64_18():
    # 12-real FP64 storage rebuilds row 2 with the same cross product that
    # reunitarisation used to write it, so it loses nothing: the FP64-12
    # chain equals the FP64-18 chain bit for bit (heatbath, overrelaxation,
    # measurement)
    a = su3hb.Lattice([8, 6, 4, 4], seed=44, precision=su3hb.FP64_18)
    b = su3hb.Lattice([8, 6, 4, 4], seed=44, precision=su3hb.FP64_12)
    assert np.array_equal(a.get_links(), b.get_links())
    sa = a.sweep_measure(5.8, n_hit=8, n_sweeps=3)
    sb = b.sweep_measure(5.8, n_hit=8, n_sweeps=3)
    a.overrelax(5.8, n_sweeps=2)
    b.overrelax(5.8, n_sweeps=2)
    a.sweep(5.8, n_hit=8, n_sweeps=2)
    b.sweep(5.8, n_hit=8, n_sweeps=2)
    assert np.array_equal(a.get_links(), b.get_links())
    assert np.array_equal(sa, sb, equal_nan=True)


def test_resume_is_bitwise(oracle_mod):
    a = su3hb.Lattice([8, 4, 4, 4], seed=21)
    a.sweep(5.8, n_hit=8, n_sweeps=6)
    b = su3hb.Lattice([8, 4, 4, 4], seed=21)
    b.sweep(5.8, n_hit=8, n_sweeps=2)
    links, (seed, sw) = b.get_links(), b.get_state()
    c = su3hb.Lattice([8, 4, 4, 4], seed=999, start=su3hb.COLD)
    c.set_links(links)
    c.set_state(seed, sw)
    c.sweep(5.8, n_hit=8, n_sweeps=4)
    assert np.array_equal(a.get_links(), c.get_links())
    assert c.get_state() == (21, 6)


@pytest.mark.parametrize("prec,ext", [(su3hb.FP64_18, [12, 6, 4, 8]), (su3hb.FP32_12, [12, 6, 4, 8]),
                                      (su3hb.FP32_18, [8, 4, 8, 16]), (su3hb.FP64_18, [16, 8, 4, 16]),
                                      (su3hb.FP64_12, [16, 8, 4, 16])])
def test_launch_shape_invariance(prec, ext):
    # every block size, block order and occupancy target gives the same links
    ref = None
    used7 = set()
    fp32 = prec in (su3hb.FP32_18, su3hb.FP32_12)
    for waves in ((2, 3, 4) if fp32 else (2, 3)):
        for block in (64, 128, 256):
            for order in range(32):
                g = su3hb.Lattice(ext, seed=8, precision=prec)
                g.set_launch(block, order, waves)
                b, o, w = g.get_launch()
                # + 8: alternate slices walk backwards; + 16: waves stage
                # U_mu neighbours in LDS (not with order 7); an order that
                # does not apply falls back to 1 or 2 and keeps the flags
                assert (b, w) == (block, waves) and o & 8 == order & 8
                assert o & 16 == (order & 16 if o & 7 != 7 else 0)
                assert o & 7 == order & 7 or o & 7 in (1, 2)
                if order & 7 == 7 and o & 7 == 7:
                    used7.add(block)
                series = g.sweep_measure(6.1, n_hit=8, n_sweeps=2)
                links = g.get_links()
                if ref is None:
                    ref, ref_series = links, series
                assert np.array_equal(links, ref), (block, order, waves)
                # the fused measurement sums per block: other block sizes
                # group the sum differently
                assert np.allclose(series, ref_series, rtol=1e-12, atol=0, equal_nan=True), (block, order, waves)
    if ext[0] % 16 == 0 and ext[3] % 16 == 0:
        assert used7, "the 4D wave-tile order was never in effect"
    with pytest.raises(su3hb.SU3HBError):
        g.set_launch(96, 0, 2)
    if not fp32:
        with pytest.raises(su3hb.SU3HBError):
            g.set_launch(64, 0, 4)
    with pytest.raises(su3hb.SU3HBError):
        g.set_launch(64, 32, 2)


@pytest.mark.parametrize("prec,ext", [(su3hb.FP64_18, [48, 8, 4, 4]), (su3hb.FP32_12, [48, 8, 4, 4]),
                                      (su3hb.FP32_18, [10, 6, 4, 2]), (su3hb.FP64_12, [6, 10, 4, 2]),
                                      (su3hb.FP64_18, [14, 6, 4]), (su3hb.FP32_12, [26, 22]),
                                      (su3hb.FP64_18, [6, 4, 4, 2, 4])])
def test_staged_neighbours_bit_identical(prec, ext):
    # waves that stage the U_mu links of the planes nu = 0, 1 in LDS give the
    # links, counters and fused plaquettes of the unstaged launch, also with
    # ragged last waves, row wraps inside a wave and wraps along direction 1
    ref = su3hb.Lattice(ext, seed=12, precision=prec)
    ref.set_launch(128, 1, 2)
    ref_series, ref_stats = ref.sweep_measure(5.9, n_hit=8, n_sweeps=3, stats=True)
    staged = 0
    for block in (64, 128, 256):
        for order in (16, 17, 25, 18, 21, 22):
            g = su3hb.Lattice(ext, seed=12, precision=prec)
            g.set_launch(block, order, 2)
            if not g.get_launch()[1] & 16:
                continue
            staged += 1
            series, stats = g.sweep_measure(5.9, n_hit=8, n_sweeps=3, stats=True)
            assert np.array_equal(g.get_links(), ref.get_links()), (block, order)
            if block == 128 and order & 7 in (0, 1, 2, 4):  # the same links per block
                assert np.array_equal(series, ref_series, equal_nan=True), (block, order)
            assert np.allclose(series, ref_series, rtol=1e-12, atol=0, equal_nan=True), (block, order)
            # counters exact; the running action change is a per-block sum
            assert {k: v for k, v in stats.items() if k != "dtrace"} == \
                {k: v for k, v in ref_stats.items() if k != "dtrace"}, (block, order)
            assert stats["dtrace"] == pytest.approx(ref_stats["dtrace"], rel=1e-12, abs=1e-9)
    assert staged >= 6


def test_staging_beyond_lds_is_refused():
    # a 4096 x 4 torus stages 64 + 4096 links per wave: far beyond the LDS of
    # a block, so the shape is refused and the launch stays as it was
    g = su3hb.Lattice([4096, 4], seed=3, precision=su3hb.FP64_18)
    g.set_launch(128, 1, 2)
    with pytest.raises(su3hb.SU3HBError) as ei:
        g.set_launch(128, 17, 2)
    assert ei.value.code == su3hb.EUNSUPPORTED and "LDS" in str(ei.value)
    assert g.get_launch() == (128, 1, 2)
    g.sweep(6.0, n_hit=8, n_sweeps=1)  # still usable


def test_graph_replay_equals_direct_launches():
    # graph replays (su3hb_sweep) against kernel-by-kernel launches
    # (su3hb_sweep_timed), with eager work and synchronisation in between
    a = su3hb.Lattice([8, 8, 4, 4], seed=31)
    b = su3hb.Lattice([8, 8, 4, 4], seed=31)
    for k in range(4):
        sa = a.sweep_measure(5.9, n_hit=8, n_sweeps=2)
        _, sb = b.sweep_timed(5.9, n_hit=8, n_sweeps=2, measure=True)
        assert np.array_equal(a.get_links(), b.get_links()), k
        assert np.array_equal(sa, sb, equal_nan=True), k
        a.plaquette(5.9)
    assert a.get_state() == b.get_state() == (31, 8)


def test_running_trace_matches_recompute():
    g = su3hb.Lattice([8, 8, 8, 4], seed=4)
    t0 = g.plaquette(5.7)[5]
    st = g.sweep(5.7, n_hit=8, n_sweeps=10, stats=True)
    t1 = g.plaquette(5.7)[5]
    say(f"  running trace {t0 + st['dtrace']:.12f} vs recomputed {t1:.12f}")
    assert abs(t0 + st["dtrace"] - t1) < 1e-11 * abs(t1)
    assert st["link_updates"] == 10 * 2048 * 4


@pytest.mark.parametrize("prec", [su3hb.FP64_18, su3hb.FP32_18])
def test_batch_replica_equals_single(prec):
    reps = [((8, 8, 8, 8), 5.7, 101, su3hb.HOT), ((6, 4, 4, 2), 6.3, 202, su3hb.HOT),
            ((4, 4, 4, 4), 5.5, 303, su3hb.COLD)]
    b0 = su3hb.Batch(4, reps, precision=prec)
    b1 = su3hb.Batch(4, reps, precision=prec)
    b0.sweep(n_hit=8, n_sweeps=3, mode=0)
    b1.sweep(n_hit=8, n_sweeps=3, mode=1)      # persistent cooperative launch
    pb = b0.plaquette()
    for r, (ext, beta, seed, start) in enumerate(reps):
        s = su3hb.Lattice(ext, precision=prec, start=start, seed=seed)
        s.sweep(beta, n_hit=8, n_sweeps=3)
        ls = s.get_links()
        assert np.array_equal(b0.get_links(r), ls), r
        assert np.array_equal(b1.get_links(r), ls), r
        assert np.allclose(pb[r], s.plaquette(beta), rtol=1e-14, atol=0, equal_nan=True)


def test_persistent_batch_larger_than_grid():
    # 40 replicas of 12^4: 840 persistent blocks of 512 links, more than one
    # per resident block, so every block loops over several logical blocks
    # between grid barriers; two persistent calls equal one per-slice call
    # of twice the sweeps, bit for bit, with the same counters
    reps = [((12, 12, 12, 12), 5.5 + 0.025 * r, 1000 + r, su3hb.HOT) for r in range(40)]
    b0 = su3hb.Batch(4, reps, precision=su3hb.FP32_18)
    b1 = su3hb.Batch(4, reps, precision=su3hb.FP32_18)
    s0 = b0.sweep(n_hit=8, n_sweeps=4, mode=0, stats=True)
    s1a = b1.sweep(n_hit=8, n_sweeps=2, mode=1, stats=True)
    s1b = b1.sweep(n_hit=8, n_sweeps=2, mode=1, stats=True)
    for r in (0, 17, 39):
        assert np.array_equal(b0.get_links(r), b1.get_links(r)), r
    for k in ("attempts", "accepts"):
        assert list(s0[k]) == [a + b for a, b in zip(s1a[k], s1b[k])], k
    assert s0["link_updates"] == s1a["link_updates"] + s1b["link_updates"] == 4 * 40 * 4 * 12 ** 4
    assert np.allclose(b0.plaquette(), b1.plaquette(), rtol=0, atol=0, equal_nan=True)


@pytest.mark.parametrize("ext,prec,tol", [([8, 8, 8, 8], su3hb.FP64_18, 1e-13), ([6, 4, 8], su3hb.FP64_18, 1e-13),
                                          ([8, 8, 8, 8], su3hb.FP64_12, 1e-13),
                                          ([16, 8], su3hb.FP64_18, 1e-13), ([4, 4, 2, 4, 2], su3hb.FP64_18, 1e-13),
                                          ([8, 8, 8, 8], su3hb.FP32_12, 2e-6), ([8, 8, 8, 8], su3hb.FP32_18, 2e-6)])
def test_fused_measurement_equals_plaquette_kernel(ext, prec, tol):
    # sweep_measure measures a single-layer lattice inside the parity-1
    # update slices; the standalone kernel measures the links afterwards
    a = su3hb.Lattice(ext, seed=17, precision=prec)
    b = su3hb.Lattice(ext, seed=17, precision=prec)
    beta = 5.9
    fused = a.sweep_measure(beta, n_hit=8, n_sweeps=5)
    sep = []
    for _ in range(5):
        b.sweep(beta, n_hit=8, n_sweeps=1)
        sep.append(b.plaquette(beta))
    sep = np.array(sep)
    assert np.array_equal(a.get_links(), b.get_links())
    assert np.array_equal(np.isnan(fused), np.isnan(sep))
    good = ~np.isnan(sep)
    d = np.abs(fused[good] - sep[good]) / np.maximum(1.0, np.abs(sep[good]))
    say(f"  fused vs kernel max rel diff = {d.max():.3e}")
    assert d.max() <= tol


@pytest.mark.parametrize("prec,tol", [(su3hb.FP64_18, TOL64), (su3hb.FP32_18, TOL32), (su3hb.FP32_12, TOL32)])
@pytest.mark.parametrize("mode", [0, 1])
def test_batch_replicas_match_oracle(oracle_mod, prec, tol, mode):
    # a mixed batch (own extents, couplings, seeds and starts per replica):
    # every replica after one batched sweep equals the oracle run on that
    # replica alone, link by link, with the integer counters summed over the
    # replicas bit-exact; mode 0 replays per-slice launches, mode 1 is the
    # persistent launch.  FP32 storage starts the oracle from the FP32-rounded
    # links the GPU holds.
    reps = [((8, 8, 8, 8), 5.7, 101, su3hb.HOT), ((6, 4, 4, 2), 6.3, 202, su3hb.HOT),
            ((4, 4, 4, 4), 5.5, 303, su3hb.COLD), ((12, 6, 4, 8), 6.05, 404, su3hb.HOT)]
    say(f"case batch of {len(reps)} prec={prec} mode={mode}")
    b = su3hb.Batch(4, reps, precision=prec)
    oracles = []
    for r, (ext, beta, seed, start) in enumerate(reps):
        o = oracle_mod.Lattice(list(ext), seed=seed, threads=8)
        if start == su3hb.COLD:
            o.cold_start()
        else:
            o.hot_start()
        if prec == su3hb.FP64_18:
            assert maxdiff(b.get_links(r), o.get_links()) <= 1e-12, r
        else:
            o.set_links(b.get_links(r))
        oracles.append(o)
    st_b = b.sweep(n_hit=8, n_sweeps=1, mode=mode, stats=True)
    att = np.zeros(3, dtype=np.int64)
    acc = np.zeros(3, dtype=np.int64)
    worst = 0.0
    for r, (ext, beta, seed, start) in enumerate(reps):
        st_o = oracles[r].sweep(beta, nhit=8, nsweeps=1)
        att += np.array(st_o["attempts"])
        acc += np.array(st_o["accepts"])
        d = maxdiff(b.get_links(r), oracles[r].get_links())
        say(f"  replica {r} {ext} beta={beta}: max |dU| = {d:.3e}")
        worst = max(worst, d)
    assert worst <= tol
    assert list(st_b["attempts"]) == list(att)
    assert list(st_b["accepts"]) == list(acc)
    assert st_b["link_updates"] == sum(4 * int(np.prod(e)) for e, *_ in reps)
    # per-replica plaquettes of the batch against the oracle's
    pb = b.plaquette()
    for r, (ext, beta, seed, start) in enumerate(reps):
        po = oracles[r].plaquette(beta)
        rt = 1e-12 if prec == su3hb.FP64_18 else 1e-5
        assert np.allclose(pb[r][[0, 1, 2, 5]], po[[0, 1, 2, 5]], rtol=rt, atol=0), r


@pytest.mark.parametrize("prec,tol", [(su3hb.FP64_18, TOL64), (su3hb.FP32_18, TOL32), (su3hb.FP32_12, TOL32),
                                      (su3hb.FP64_12, TOL64)])
@pytest.mark.parametrize("block", [64, 256])
def test_double_layered_multiblock_matches_oracle(oracle_mod, prec, tol, block):
    # a double-layered torus glued in every direction with beta0 != beta1 on
    # a lattice whose slices span several blocks: 2 x 720 links per slice,
    # 720 not a multiple of 64 (the last tile of each slab is partial) nor of
    # the block, so the layer boundary falls inside a block.  Per link after
    # one sweep from a shared start (FP32: the GPU's rounded start), the
    # running action, the counters, and the fused two-layer measurement of a
    # second sweep against the oracle's plaquettes of the same links.
    ext, b0, b1 = [6, 10, 6, 4], 5.5, 6.2
    g, o = pair(oracle_mod, ext, nlat=2, mask=0b1111, prec=prec, seed=17)
    g.set_launch(block, 1, 2)
    if prec != su3hb.FP64_18:
        o.set_links(g.get_links())
    st_g = g.sweep(b0, b1, n_hit=8, n_sweeps=1, stats=True)
    st_o = o.sweep(b0, b1, nhit=8, nsweeps=1)
    d = maxdiff(g.get_links(), o.get_links())
    say(f"  DLT {ext} block={block} prec={prec}: max |dU| after 1 sweep = {d:.3e}")
    assert d <= tol
    assert list(st_g["attempts"]) == list(st_o["attempts"])
    assert list(st_g["accepts"]) == list(st_o["accepts"])
    rel = 1e-9 if prec in (su3hb.FP64_18, su3hb.FP64_12) else 1e-4
    assert abs(st_g["dtrace"] - st_o["dtrace"]) <= rel * max(1.0, abs(st_o["dtrace"]))
    # second sweep measured inside the update (three LDS classes), compared
    # with the oracle's measurement of the GPU's resulting links
    series = g.sweep_measure(b0, b1, n_hit=8, n_sweeps=1)
    o.set_links(g.get_links())
    po = o.plaquette(b0, b1)
    rt = 1e-12 if prec in (su3hb.FP64_18, su3hb.FP64_12) else 2e-6
    say(f"  fused measurement {series[0]} oracle {po}")
    assert np.allclose(series[0], po, rtol=rt, atol=0, equal_nan=True)
