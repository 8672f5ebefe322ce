"""Long GPU runs against exact results and the paper's statistics.

Error bars are 32-bin jackknife errors of the per-sweep plaquette series;
comparisons use the Gaussian difference test of the paper (Sec. 3.2): two
estimates agree when Q = erfc(|m1-m2| / sqrt(2 (e1^2 + e2^2))) is not tiny.
Every run is seeded, so each test is deterministic.
"""
import json
import os
import sys

import numpy as np
import pytest

import paper_0904_0642_amd as su3hb
from paper_0904_0642_amd import workloads
from exact_su3 import dlt_two_coupling_exact, u_exact
from stats import gaussian_difference_q, jackknife_mean, tau_int

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
QMIN = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    su3hb.lib()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_series(lat, beta0, beta1=None, n_hit=8, ntherm=200, nmeas=4000, col=0):
    lat.sweep(beta0, beta1, n_hit=n_hit, n_sweeps=ntherm)
    s = lat.sweep_measure(beta0, beta1, n_hit=n_hit, n_sweeps=nmeas)
    return s[:, col] if isinstance(col, int) else s[:, col]


def test_2d_32x32_exact():
    # D = 2 torus 32^2 at beta = 4: <P> = u(4) = 0.27961914940930...
    lat = su3hb.Lattice([32, 32], seed=1)
    s = run_series(lat, 4.0, ntherm=200, nmeas=20000)
    m, e = jackknife_mean(s, 32)
    say(f"  2D 32^2 beta=4: <P> = {m:.6f} +- {e:.6f}, exact {u_exact(4.0):.6f}")
    assert gaussian_difference_q(m, e, u_exact(4.0), 0.0) > QMIN


def test_2d_heatbath_with_overrelaxation_exact():
    # one heatbath sweep and two overrelaxation sweeps per measurement leave
    # the Boltzmann distribution in place: <P> = u(4) on 32^2
    lat = su3hb.Lattice([32, 32], seed=11)
    for _ in range(200):
        lat.sweep(4.0, n_hit=8, n_sweeps=1)
        lat.overrelax(4.0, n_sweeps=2)
    s = []
    for _ in range(8000):
        lat.sweep(4.0, n_hit=8, n_sweeps=1)
        lat.overrelax(4.0, n_sweeps=2)
        s.append(lat.plaquette(4.0)[0])
    m, e = jackknife_mean(np.array(s), 32)
    say(f"  2D 32^2 beta=4 HB+2OR: <P> = {m:.6f} +- {e:.6f}, exact {u_exact(4.0):.6f}")
    assert gaussian_difference_q(m, e, u_exact(4.0), 0.0) > QMIN


@pytest.mark.parametrize("mask", [0b11, 0b01])
def test_2d_double_layered_exact(mask):
    lat = su3hb.Lattice([16, 16], nlat=2, dlt_mask=mask, seed=2)
    s = run_series(lat, 4.0, ntherm=200, nmeas=10000)
    m, e = jackknife_mean(s, 32)
    say(f"  2D DLT mask={mask:02b} beta=4: <P> = {m:.6f} +- {e:.6f}")
    assert gaussian_difference_q(m, e, u_exact(4.0), 0.0) > QMIN


def test_2d_double_layered_two_couplings_exact():
    # beta0 != beta1: per-layer averages and the beta-weighted sum against
    # the exact 2D values (each plaquette at its own coupling, tag rule)
    b0, b1 = 4.0, 2.0
    lat = su3hb.Lattice([16, 16], nlat=2, dlt_mask=0b11, seed=12)
    lat.sweep(b0, b1, n_hit=8, n_sweeps=200)
    rows = lat.sweep_measure(b0, b1, n_hit=8, n_sweeps=4000)[:, [3, 4, 5]]
    exact = dlt_two_coupling_exact(16, 16, b0, b1)
    for k, name in enumerate(("layer 0", "layer 1", "weighted sum")):
        m, e = jackknife_mean(rows[:, k], 32)
        q = gaussian_difference_q(m, e, exact[k], 0.0)
        say(f"  2D DLT beta=({b0},{b1}) {name}: {m:.6f} +- {e:.6f}, exact {exact[k]:.6f}, Q={q:.2f}")
        assert q > QMIN


def test_4d_strong_coupling():
    lat = su3hb.Lattice([8, 8, 8, 8], seed=3)
    s = run_series(lat, 1.0, ntherm=100, nmeas=3000)
    m, e = jackknife_mean(s, 32)
    say(f"  4D beta=1: <P> = {m:.6f} +- {e:.6f}, u(1) = {u_exact(1.0):.6f}")
    assert gaussian_difference_q(m, e, u_exact(1.0), 2e-6) > QMIN


def test_paper_4x4x4x4_beta5p6_ordered():
    # Sec. 3.2: 4^4, beta = 5.6, ordered start, (1STAT) statistics:
    # act = 0.53770(18) single-processor, 0.53811(19) MPI
    ref = GOLDEN["pbc_4x4x4x4_b5.6_ordered"]
    st = GOLDEN["statistics_1STAT"]
    lat = su3hb.Lattice(ref["extents"], start=su3hb.COLD, seed=5)
    lat.sweep(ref["beta"], n_hit=1, n_sweeps=st["nequi"])
    s = lat.sweep_measure(ref["beta"], n_hit=1, n_sweeps=st["nrpt"] * st["nmeas"] * st["nsw"])[:, 0]
    m, e = jackknife_mean(s, 32)
    q1 = gaussian_difference_q(m, e, *ref["act_single"])
    q2 = gaussian_difference_q(m, e, *ref["act_mpi"])
    say(f"  4^4 beta=5.6: act = {m:.5f}({e*1e5:.0f}); paper {ref['act_single']} Q={q1:.2f}, {ref['act_mpi']} Q={q2:.2f}")
    # integrated autocorrelation time, per sweep and per measurement every nsw sweeps
    t1, dt1, w1 = tau_int(s)
    t2, dt2, w2 = tau_int(s[:: st["nsw"]])
    say(f"  tau_int = {t1:.1f}({dt1:.1f}) sweeps (window {w1}), {t2:.1f}({dt2:.1f}) measurements every "
        f"{st['nsw']} sweeps; the paper estimates 49.5(3.4)")
    # the paper's estimate is in units of sweeps (reading R-TAU)
    assert gaussian_difference_q(t1, dt1, *ref["tau_int"]) > QMIN
    assert max(q1, q2) > QMIN


def full_statistics():
    # eq. (1STAT): nequi sweeps, then nrpt * nmeas * nsw sweeps (measured
    # here after every sweep)
    st = GOLDEN["statistics_1STAT"]
    return st["nequi"], st["nrpt"] * st["nmeas"] * st["nsw"]


def test_paper_table1_8x8x8x4():
    ref = GOLDEN["pbc_8x8x8x4_b5.65"]
    lat = su3hb.Lattice(ref["extents"], start=su3hb.COLD, seed=6)
    ntherm, nmeas = full_statistics()
    s = run_series(lat, ref["beta"], n_hit=1, ntherm=ntherm, nmeas=nmeas)
    m, e = jackknife_mean(s, 32)
    qs = [gaussian_difference_q(m, e, *v) for v in ref["actm"]]
    say(f"  8^3 4 beta=5.65: act = {m:.6f}({e*1e6:.0f}); Q vs Table 1 rows = {[round(q, 2) for q in qs]}")
    assert qs[0] > QMIN


def test_paper_table2_16x16x16x4():
    ref = GOLDEN["pbc_16x16x16x4_b5.65"]
    lat = su3hb.Lattice(ref["extents"], start=su3hb.COLD, seed=7)
    ntherm, nmeas = full_statistics()
    lat.sweep(ref["beta"], n_hit=1, n_sweeps=ntherm)
    ser = lat.sweep_measure(ref["beta"], n_hit=1, n_sweeps=nmeas)
    ms, es = jackknife_mean(ser[:, 1], 32)
    mt, et = jackknife_mean(ser[:, 2], 32)
    qs = gaussian_difference_q(ms, es, *ref["spacelike_single"])
    qt = gaussian_difference_q(mt, et, *ref["timelike_single"])
    say(f"  16^3 4 beta=5.65: spacelike {ms:.6f}({es*1e6:.0f}) Q={qs:.2f}; timelike {mt:.6f}({et*1e6:.0f}) Q={qt:.2f}")
    assert qs > QMIN and qt > QMIN


def test_paper_table3_dlt_8x8x8x4():
    ref = GOLDEN["dlt_8x8x8x4_b5.55_disordered"]
    lat = su3hb.Lattice(ref["extents"], nlat=2, dlt_mask=0b1111, start=su3hb.HOT, seed=8)
    ntherm, nmeas = full_statistics()
    s = run_series(lat, ref["beta"], n_hit=1, ntherm=ntherm, nmeas=nmeas)
    m, e = jackknife_mean(s, 32)
    qs = [gaussian_difference_q(m, e, *v) for v in ref["actm"]]
    say(f"  DLT 8^3 4 beta=5.55: act = {m:.6f}({e*1e6:.0f}); Q vs Table 3 rows = {[round(q, 2) for q in qs]}")
    assert max(qs) > QMIN


def test_batched_fp32_replicas_reproduce_table1():
    # the batched form: 64 independent FP32-18 replicas of the Table 1 lattice
    # (8^3 4, beta = 5.65, ordered starts, own seeds) in one batch; the
    # replica means are independent, so their spread gives the error of the
    # ensemble mean, compared with the FP64 numbers of Table 1
    ref = GOLDEN["pbc_8x8x8x4_b5.65"]
    nrep = 64
    seeds = workloads.seeds(nrep, seed=2024)
    reps = [(tuple(ref["extents"]), ref["beta"], sd, su3hb.COLD) for sd in seeds]
    b = su3hb.Batch(4, reps, precision=su3hb.FP32_18)
    b.sweep(n_hit=1, n_sweeps=1000, mode=0)
    acc = np.zeros(nrep)
    nmeas = 1000
    for _ in range(nmeas):
        b.sweep(n_hit=1, n_sweeps=2, mode=0)
        acc += b.plaquette()[:, 0]
    means = acc / nmeas
    m, e = means.mean(), means.std(ddof=1) / np.sqrt(nrep)
    qs = [gaussian_difference_q(m, e, *v) for v in ref["actm"]]
    say(f"  batch of {nrep} FP32 replicas 8^3 4 beta=5.65: act = {m:.6f}({e*1e6:.0f}); "
        f"Q vs Table 1 rows = {[round(q, 2) for q in qs]}")
    assert qs[0] > QMIN


def test_long_run_gpu_vs_oracle(oracle_mod):
    # 4^4, beta = 6.0, ordered start, n_hit = 8 (the small workload): the GPU
    # chain and an independent oracle chain (other seed) agree statistically
    lat = su3hb.Lattice([4, 4, 4, 4], start=su3hb.COLD, seed=1)
    sg = run_series(lat, 6.0, ntherm=500, nmeas=32000)
    mg, eg = jackknife_mean(sg, 32)
    o = oracle_mod.Lattice([4, 4, 4, 4], seed=2)
    o.cold_start()
    o.sweep(6.0, nhit=8, nsweeps=500)
    so = []
    for _ in range(4000):
        o.sweep(6.0, nhit=8, nsweeps=1)
        so.append(o.plaquette(6.0)[0])
    mo, eo = jackknife_mean(np.array(so), 32)
    q = gaussian_difference_q(mg, eg, mo, eo)
    say(f"  4^4 beta=6: GPU {mg:.5f}({eg*1e5:.0f}) oracle {mo:.5f}({eo*1e5:.0f}) Q={q:.2f}")
    # two combined jackknife error bars
    assert abs(mg - mo) < 2 * np.hypot(eg, eo)


def test_acceptance_near_97_percent():
    # Sec. 2.1 puts the single-hit acceptance near 97% at the couplings of interest
    lat = su3hb.Lattice([16, 16, 16, 16], seed=9)
    lat.sweep(6.0, n_hit=1, n_sweeps=100)
    st = lat.sweep(6.0, n_hit=1, n_sweeps=20, stats=True)
    acc = np.array(st["accepts"]) / np.array(st["attempts"])
    say(f"  16^4 beta=6.0 1-hit acceptance per subgroup: {acc}")
    assert np.all(acc > 0.95) and np.all(acc < 0.995)


def test_fp32_vs_fp64_same_plaquette():
    # FP32 link storage (FP64 heatbath, reunitarisation, accumulation) gives
    # the same observables as FP64 within the statistical error: total,
    # spacelike and timelike plaquette and the action beta sum_p (1/3) Re Tr
    # U_p.  Each precision runs eight independent chains (seeds 10..17; the
    # same seeds for every precision, which only correlates the chains and
    # makes the test conservative), pooled as the mean of the chain means
    # with the error of that mean, so that no single reference chain's
    # fluctuation decides the comparison.
    names = ("total", "spacelike", "timelike", "action")
    cols = (0, 1, 2, 5)
    seeds = tuple(range(10, 18))
    res = {}
    for prec in (su3hb.FP64_18, su3hb.FP32_18, su3hb.FP32_12, su3hb.FP64_12):
        per = []
        for sd in seeds:
            lat = su3hb.Lattice([16, 16, 16, 16], seed=sd, precision=prec)
            lat.sweep(6.0, n_hit=8, n_sweeps=300)
            ser = lat.sweep_measure(6.0, n_hit=8, n_sweeps=4000)
            lat.close()
            per.append([jackknife_mean(ser[:, c], binned(ser[:, c])) for c in cols])
        res[prec] = [(np.mean([p[k][0] for p in per]), np.sqrt(np.sum([p[k][1] ** 2 for p in per])) / len(per))
                     for k in range(len(cols))]
    for prec in (su3hb.FP32_18, su3hb.FP32_12, su3hb.FP64_12):
        for k, name in enumerate(names):
            (m, e), (m64, e64) = res[prec][k], res[su3hb.FP64_18][k]
            say(f"  16^4 beta=6.0 prec={prec} {name}: {m:.8g}({e:.2g}) vs FP64 {m64:.8g}({e64:.2g}), "
                f"{(m - m64) / np.hypot(e, e64):+.2f} sigma")
            assert abs(m - m64) < 2 * np.hypot(e, e64)


def binned(series, nmax=32, nmin=8):
    """Jackknife bins of at least 4 tau_int sweeps each (shorter bins are
    correlated and underestimate the error), between nmin and nmax bins."""
    tau = tau_int(series)[0]
    return int(max(nmin, min(nmax, len(series) // max(1, int(np.ceil(4 * tau))))))


def pooled(chains, col):
    """Mean of the chain means of column col and the error of that mean
    (chains independent, each with its jackknife error in bins of at least
    4 tau_int)."""
    ms, es = zip(*[jackknife_mean(c[:, col], binned(c[:, col])) for c in chains])
    return float(np.mean(ms)), float(np.sqrt(np.sum(np.square(es))) / len(ms))


def test_config3_double_layered_fp32_error_per_observable(oracle_mod):
    # two 24^3 x 8 layers glued in every direction, beta = 5.69, hot starts,
    # per observable (total, spacelike, timelike, layer 0, layer 1, the
    # beta-weighted action).  FP64 reference: the oracle's chain from seed 1,
    # 500 sweeps as the workload states, and four FP64-18 GPU chains (seeds
    # 1..4, 2200 sweeps each).  FP32-18 and FP32-12 storage (FP64
    # Kennedy-Pendleton draw, reunitarisation and accumulation) run the same
    # four seeds.  Pooled over the four chains (first 200 sweeps
    # thermalisation), each FP32 form is compared with FP64 within two
    # combined jackknife errors (bins of at least 4 tau_int).  The FP64 pool
    # is compared with the oracle's 500-sweep chain (first 100 sweeps
    # thermalisation) by the paper's Gaussian difference test (Q > 1e-3, as
    # for the paper's tables): that chain has about 20 independent
    # measurements, too few for a two-error bound on many observables.
    ext, beta, ntherm = (24, 24, 24, 8), 5.69, 200
    names = ("total", "spacelike", "timelike", "layer 0", "layer 1", "action")
    o = oracle_mod.Lattice(list(ext), nlat=2, dlt_mask=0b1111, seed=1, threads=16)
    o.hot_start()
    ser_o = []
    for _ in range(500):
        o.sweep(beta, nhit=8, nsweeps=1)
        ser_o.append(o.plaquette(beta))
    ser_o = np.array(ser_o)[100:]
    chains = {}
    for prec in (su3hb.FP64_18, su3hb.FP32_18, su3hb.FP32_12):
        chains[prec] = []
        for seed in (1, 2, 3, 4):
            lat = su3hb.Lattice(ext, nlat=2, dlt_mask=0b1111, precision=prec, seed=seed)
            chains[prec].append(lat.sweep_measure(beta, n_hit=8, n_sweeps=ntherm + 2000)[ntherm:])
            lat.close()
    for k, name in enumerate(names):
        m64, e64 = pooled(chains[su3hb.FP64_18], k)
        mo, eo = jackknife_mean(ser_o[:, k], binned(ser_o[:, k]))
        z = (m64 - mo) / np.hypot(e64, eo)
        q = gaussian_difference_q(m64, e64, mo, eo)
        say(f"  2x24^3x8 beta={beta} {name}: FP64 GPU pool {m64:.8g}({e64:.2g}) vs oracle chain "
            f"{mo:.8g}({eo:.2g}), {z:+.2f} sigma, Q = {q:.2f}")
        assert q > QMIN, ("oracle", name)
        for prec in (su3hb.FP32_18, su3hb.FP32_12):
            m, e = pooled(chains[prec], k)
            z = (m - m64) / np.hypot(e, e64)
            say(f"    prec={prec}: {m:.8g}({e:.2g}), {(m - m64):+.2e} = {z:+.2f} sigma against FP64")
            assert abs(z) < 2.0, (prec, name)


@pytest.mark.parametrize("beta", [5.7, 6.0])
def test_config2_trajectory_and_first_flip(oracle_mod, beta):
    # 16^4, hot start from seed 1, 200 sweeps with the plaquette after every
    # sweep, GPU against the oracle from the same start and random numbers.
    # The chains differ by rounding (libm against device functions, FMA
    # contraction); that difference grows smoothly from sweep to sweep until
    # it flips an accept/reject decision (Sec. 3), which moves a link by far
    # more than the smooth growth.  The first sweep whose largest link
    # difference jumps (to more than 1e-4 and 30 times the sweep before) or
    # whose counters differ is replayed on the oracle slice by slice from the
    # oracle's own configuration; in the first slice whose output differs from
    # the GPU's by more than that jump threshold every such link is a flipped
    # decision, printed with its distance from the acceptance threshold
    # |R4^2 - (1 - delta/2)|, which must be within the perturbation the
    # smooth difference can cause.  Over the run the mean plaquettes agree
    # within two combined jackknife error bars.
    ext, nsw, ntherm = (16, 16, 16, 16), 200, 50
    g = su3hb.Lattice(ext, seed=1)
    o = oracle_mod.Lattice(list(ext), seed=1, threads=16)
    o.hot_start()
    first = None
    pg, po, dmax = [], [], []
    prev_o = o.get_links()
    for k in range(nsw):
        st_g = g.sweep(beta, n_hit=8, n_sweeps=1, stats=True)
        st_o = o.sweep(beta, nhit=8, nsweeps=1)
        pg.append(g.plaquette(beta)[0])
        po.append(o.plaquette(beta)[0])
        if first is None:
            cur_g, cur_o = g.get_links(), o.get_links()
            dmax.append(float(np.abs(cur_g - cur_o).max()))
            before = dmax[-2] if len(dmax) > 1 else 0.0
            same = (list(st_g["attempts"]) == list(st_o["attempts"])
                    and list(st_g["accepts"]) == list(st_o["accepts"]))
            jump = dmax[-1] > 1e-4 and dmax[-1] > 30.0 * before
            if jump or not same:
                first = (k, prev_o, cur_g, before)
            prev_o = cur_o
    pg, po = np.array(pg), np.array(po)
    say(f"  16^4 beta={beta}: max |dU| GPU vs oracle after each sweep: "
        f"{' '.join(f'{d:.1e}' for d in dmax)}")
    say(f"  per-sweep |d<P>| max over the first 10 sweeps: {np.abs(pg[:10] - po[:10]).max():.2e}")
    if first is None:
        say(f"  no accept/reject decision differs in {nsw} sweeps")
    else:
        k, before_o, after_g, dprev = first
        thr = max(1e-4, 30.0 * dprev)
        par = np.zeros(int(np.prod(ext)), dtype=np.int64)
        idx = np.arange(par.size)
        stride = 1
        for n in ext:
            par += (idx // stride) % n
            stride *= n
        par &= 1
        o2 = oracle_mod.Lattice(list(ext), seed=1, threads=16)
        o2.set_links(before_o)
        o2.sweep_counter = k
        flips = []
        for p in (0, 1):
            for mu in range(4):
                state = o2.get_links()
                o2.update_slice(p, mu, beta, nhit=8)
                res = o2.get_links()
                sites = np.flatnonzero(par == p)
                dd = np.abs(res[0, sites, mu] - after_g[0, sites, mu]).reshape(len(sites), -1).max(axis=1)
                if (dd > thr).any():
                    o2.set_links(state)
                    for s, d in zip(sites[dd > thr], dd[dd > thr]):
                        flips.append((p, mu, int(s), float(d), o2.link_margin(0, int(s), mu, beta, nhit=8)))
                    break
            if flips:
                break
        say(f"  sweep {k}: first decision flip; largest smooth difference before it {dprev:.1e}; flipped links "
            f"(parity, mu, site, |dU|, |R4^2 - (1 - delta/2)|) = {[tuple(f'{v:.3g}' if isinstance(v, float) else v for v in f) for f in flips[:4]]}")
        assert flips, "a jump in the chains' difference without a flipped link"
        # the flipped decisions lay within reach of the smooth difference
        assert min(f[4] for f in flips) < max(1e-9, 1e3 * dprev)
    mg, eg = jackknife_mean(pg[ntherm:], 15)
    mo, eo = jackknife_mean(po[ntherm:], 15)
    say(f"  <P> over sweeps {ntherm}..{nsw}: GPU {mg:.6f}({eg*1e6:.0f}) oracle {mo:.6f}({eo*1e6:.0f})")
    assert abs(mg - mo) < 2 * np.hypot(eg, eo) or abs(mg - mo) < 1e-9
