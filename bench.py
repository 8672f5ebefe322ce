#!/usr/bin/env python3
"""Benchmark: checkerboard Cabibbo-Marinari / FHKP SU(3) heatbath sweeps on one MI355X.

A step is one sweep of the whole hot path -- 2D checkerboard slice updates
(staple, three SU(2) subgroup heatbaths in multi-hit form, reunitarisation,
fused action bookkeeping) followed by the plaquette measurement -- on a
resident lattice.  Default workload: D = 4, 48^4 periodic torus, beta = 6.2,
FP64 links (18 reals), disordered (Haar) start from seed 1, n_hit = 8; the
FP32 12-real form is run beside it on a 64^4 lattice of about the same size
in HBM.  Inputs are synthetic (the start is drawn from the Philox stream).

Prints one JSON line.  `value` is link updates per second over the timed
sweeps; `roofline` prices the slice-update kernel against 8 TB/s with the
algorithmic bytes per launch (2D+1) * bytes_per_link * V/2 (one read of every
link of the lattice, one write of the updated half-direction), divided by the
kernel's average duration measured with HIP events around each launch.
`roofline.traffic` is the memory-side bytes per launch that rocprofv3
counter runs (FETCH_SIZE, WRITE_SIZE, scaled by a copy of known size)
recorded for this kernel source in the launch shape in effect, else null.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_0904_0642_amd", "csrc", f)
                  for f in ("update.hip", "device_math.h", "geometry.h", "layout.h", "log_table.h")]

WORKLOADS = {
    # name: (extents, precision, beta)
    "48^4-fp64": ((48, 48, 48, 48), 0, 6.2),
    "64^4-fp32-12": ((64, 64, 64, 64), 2, 6.2),
    "64^4-fp32-18": ((64, 64, 64, 64), 1, 6.2),
    "48^4-fp64-12": ((48, 48, 48, 48), 3, 6.2),
    "16^4-fp64": ((16, 16, 16, 16), 0, 6.0),
}
PREC_NAME = {0: "fp64-18", 1: "fp32-18", 2: "fp32-12", 3: "fp64-12"}
# the paper's small runs (Sec. 3, Tables 1-3 and the D = 2 check), FP64 links:
# name: (extents, layers, glued directions, cold start, beta, sweeps)
EXTRA_LEGS = ("batch", "dlt", "precision", "overrelax", "full_size", "small_configs")
SMALL_CONFIGS = {
    "config1_4^4_cold": ((4, 4, 4, 4), 1, 0, True, 6.0, 20),
    "config2a_16^4_hot_beta5.7": ((16, 16, 16, 16), 1, 0, False, 5.7, 200),
    "config2a_16^4_hot_beta6.0": ((16, 16, 16, 16), 1, 0, False, 6.0, 200),
    "config2b_32^2_hot": ((32, 32), 1, 0, False, 4.0, 20000),
    "config3_2x24^3x8_hot": ((24, 24, 24, 8), 2, 0xF, False, 5.69, 500),
}
PREC_DTYPE = {0: "f64", 1: "f32 links + f64 heatbath", 2: "f32 (12-real) links + f64 heatbath",
              3: "f64 (12-real links)"}
BYTES_PER_LINK = {0: 144, 1: 72, 2: 48, 3: 96}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, launch) -> int | None:
    """Memory-side bytes per update launch from the committed rocprofv3
    counter runs of this workload in this launch shape (block, order, waves
    as the library reports them); None when no run covers the shape or the
    runs were taken on different kernel sources."""
    path = os.path.join(PROFILES, f"update_kernel_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    entry = rec.get("by_launch", {}).get("%d,%d,%d" % tuple(launch))
    return None if entry is None else entry.get("hbm_bytes_per_launch")


def parse_launch(text: str):
    if not text:
        return None
    b, o, w = (int(v) for v in text.split(","))
    return b, o, w


def run_leg(name: str, steps: int, warmup: int, n_hit: int, autotune_ms: int, launch=None):
    import torch

    import paper_0904_0642_amd as su3hb

    ext, prec, beta = WORKLOADS[name]
    D = len(ext)
    V = int(np.prod(ext))
    lat = su3hb.Lattice(ext, precision=prec, start=su3hb.HOT, seed=1)
    if launch is not None:
        lat.set_launch(*launch)
    elif autotune_ms > 0:
        lat.autotune(autotune_ms)
    block, order, waves = lat.get_launch()
    if warmup > 0:
        lat.sweep_measure(beta, n_hit=n_hit, n_sweeps=warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timing, series = lat.sweep_timed(beta, n_hit=n_hit, n_sweeps=steps, measure=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    secs = t1 - t0
    links_per_sweep = V * D
    rate = steps * links_per_sweep / secs
    upd_ms = timing[0] / max(timing[1], 1)
    plq_ms = timing[2] / max(timing[3], 1)
    S = BYTES_PER_LINK[prec]
    bytes_per_launch = (2 * D + 1) * S * (V // 2)
    achieved = bytes_per_launch / (upd_ms * 1e-3) / 1e9
    traffic = measured_traffic(name, (block, order, waves))
    plaq = series[:, 0]
    out = {
        "rate": rate, "secs": secs, "ms_per_step": 1e3 * secs / steps,
        "update_kernel_ms": upd_ms, "plaquette_kernel_ms": plq_ms,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "kernel": f"update_kernel<{D},{PREC_NAME[prec]}>"},
        "plaquette_first_last": [float(plaq[0]), float(plaq[-1])],
        "launch": {"block": block, "order": order, "waves": waves},
        "extents": list(ext), "precision": PREC_NAME[prec], "beta": beta, "links_per_sweep": links_per_sweep,
    }
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return out


def overrelax_leg(name: str, steps: int, warmup: int, autotune_ms: int):
    """Overrelaxation sweeps (per subgroup the reflection that keeps the local
    action) on a full-size lattice: the same loads and stores as a heatbath
    sweep without the Kennedy-Pendleton draws, priced with the same bytes."""
    import torch

    import paper_0904_0642_amd as su3hb

    ext, prec, beta = WORKLOADS[name]
    D = len(ext)
    V = int(np.prod(ext))
    lat = su3hb.Lattice(ext, precision=prec, start=su3hb.HOT, seed=1)
    if autotune_ms > 0:
        lat.autotune(autotune_ms)
    lat.sweep(beta, n_hit=8, n_sweeps=max(warmup, 1))
    lat.overrelax(beta, n_sweeps=max(warmup, 1))
    t0 = lat.plaquette(beta)[5]
    torch.cuda.synchronize()
    t = time.perf_counter()
    timing, _ = lat.sweep_timed(beta, n_hit=0, n_sweeps=steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t
    upd_ms = timing[0] / max(timing[1], 1)
    bytes_per_launch = (2 * D + 1) * BYTES_PER_LINK[prec] * (V // 2)
    achieved = bytes_per_launch / (upd_ms * 1e-3) / 1e9
    t1 = lat.plaquette(beta)[5]
    out = {"value": round(steps * V * D / secs, 1), "unit": "link updates/s", "ms_per_step": round(1e3 * secs / steps, 4),
           "update_kernel_ms": round(upd_ms, 5),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": bytes_per_launch},
           "action_relative_change": float(abs(t1 - t0) / abs(t0)),
           "launch": dict(zip(("block", "order", "waves"), lat.get_launch()))}
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return out


def batch_leg(steps: int, warmup: int, n_hit: int, autotune_ms: int, nrep: int = 128, launch=None,
              modes=("graph_per_slice", "persistent")):
    """Independent replicas of mixed sizes (8^4, 12^4, 16^3x4 round robin),
    beta uniform in [5.5, 6.5], FP32 links, one launch per slice for all
    replicas replayed from a HIP graph, and the same sweeps as one persistent
    cooperative launch."""
    import torch

    import paper_0904_0642_amd as su3hb
    from paper_0904_0642_amd import workloads

    t = workloads.replica_table(nrep, seed=7)
    reps = [(e, b, sd, st) for e, b, sd, st in zip(t.extents, t.betas, t.seeds, t.starts)]
    prec = su3hb.FP32_18
    b = su3hb.Batch(4, reps, precision=prec)
    if launch is not None:
        b.set_launch(*launch)
    elif autotune_ms > 0:
        b.autotune(autotune_ms)
    shape = su3hb.su3hb_get_launch(b._h)
    if warmup > 0:
        b.sweep(n_hit=n_hit, n_sweeps=warmup, mode=0)
    links = t.links_per_sweep
    timing, _ = su3hb.su3hb_sweep_timed(b._h, 0.0, 0.0, n_hit, steps, measure=False)
    upd_ms = timing[0] / max(timing[1], 1)
    out = {}
    for mode, label in ((0, "graph_per_slice"), (1, "persistent")):
        if label not in modes:
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.sweep(n_hit=n_hit, n_sweeps=steps, mode=mode)
        torch.cuda.synchronize()
        out[label] = steps * links / (time.perf_counter() - t0)
    plaq = b.plaquette()[:, 0]
    S = BYTES_PER_LINK[prec]
    bytes_per_launch = sum((2 * 4 + 1) * S * (int(np.prod(e)) // 2) for e in t.extents)
    achieved = bytes_per_launch / (upd_ms * 1e-3) / 1e9
    res = {"value": round(max(out.values()), 1), "unit": "link updates/s",
           "by_mode": {k: round(v, 1) for k, v in out.items()},
           "replicas": nrep, "links_per_sweep": links, "precision": PREC_NAME[prec],
           "update_kernel_ms": round(upd_ms, 5),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic(f"batch-{nrep}-{PREC_NAME[prec]}", shape),
                        "algorithmic_bytes_per_launch": bytes_per_launch},
           "plaquette_mean_over_replicas": float(np.mean(plaq)),
           "launch": dict(zip(("block", "order", "waves"), shape))}
    b.close()
    torch.cuda.empty_cache()
    return res


def dlt_leg(n_hit: int, autotune_ms: int, seeds=(1, 2, 3, 4), nmeas: int = 2000, ntherm: int = 200):
    """Double-layered torus: two 24^3 x 8 layers glued in all directions,
    beta0 = beta1 = 5.69, hot starts, plaquettes measured after every sweep,
    in FP64-18, FP32-18 and FP32-12 storage, four independent chains (seeds)
    per form of ntherm + nmeas sweeps.  Each observable (total, spacelike,
    timelike, per layer, the beta-weighted action) is pooled over the chains
    (mean of the chain means, error of that mean from the chains' jackknife
    errors in bins of at least 4 tau_int), and each FP32 form's deviation
    from FP64-18 is stated in units of the combined error; the FP64-18 path
    itself is compared with the FP64 oracle in the test suite.  The rate is
    over all timed sweeps of a form."""
    import torch

    import paper_0904_0642_amd as su3hb
    from paper_0904_0642_amd.analysis import jackknife_mean, tau_int

    def nbins(x):
        # bins of at least 4 tau_int sweeps, 8 to 32 of them
        return int(max(8, min(32, len(x) // max(1, int(np.ceil(4 * tau_int(x)[0]))))))

    def pooled(chs, c):
        ms, es = zip(*[jackknife_mean(ch[:, c], nbins(ch[:, c])) for ch in chs])
        return float(np.mean(ms)), float(np.sqrt(np.sum(np.square(es))) / len(ms))

    ext, beta = (24, 24, 24, 8), 5.69
    links = 2 * int(np.prod(ext)) * 4
    names = ("total", "spacelike", "timelike", "layer0", "layer1", "action")
    res = {"lattice": "2 x 24^3 x 8, all directions glued", "beta": beta, "chains": len(seeds),
           "sweeps_per_chain": ntherm + nmeas, "thermalisation_sweeps": ntherm, "links_per_sweep": links,
           "unit": "link updates/s"}
    chains = {}
    for prec in (su3hb.FP64_18, su3hb.FP32_18, su3hb.FP32_12):
        chains[prec], secs, launch = [], 0.0, None
        for sd in seeds:
            lat = su3hb.Lattice(ext, nlat=2, dlt_mask=0xF, precision=prec, seed=sd)
            if autotune_ms > 0:
                lat.autotune(autotune_ms)
            launch = dict(zip(("block", "order", "waves"), lat.get_launch()))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            chains[prec].append(lat.sweep_measure(beta, n_hit=n_hit, n_sweeps=ntherm + nmeas)[ntherm:])
            torch.cuda.synchronize()
            secs += time.perf_counter() - t0
            lat.close()
        torch.cuda.empty_cache()
        res[PREC_NAME[prec]] = {"value": round(len(seeds) * (ntherm + nmeas) * links / secs, 1), "launch": launch}
    ref = {k: pooled(chains[su3hb.FP64_18], c) for c, k in enumerate(names)}
    res["fp64-18"]["observables"] = {k: [round(m, 9), float(f"{e:.3g}")] for k, (m, e) in ref.items()}
    for prec in (su3hb.FP32_18, su3hb.FP32_12):
        obs, dev = {}, {}
        for c, k in enumerate(names):
            m, e = pooled(chains[prec], c)
            obs[k] = [round(m, 9), float(f"{e:.3g}")]
            dev[k] = round((m - ref[k][0]) / np.hypot(e, ref[k][1]), 2)
        res[PREC_NAME[prec]]["observables"] = obs
        res[PREC_NAME[prec]]["delta_vs_fp64_in_sigma"] = dev
        res[PREC_NAME[prec]]["rate_ratio_vs_fp64"] = round(res[PREC_NAME[prec]]["value"] / res["fp64-18"]["value"], 3)
    return res


def precision_study(n_hit: int, ntherm: int = 200, nmeas: int = 2000):
    """Equal-volume comparison at equal sweep count (hence equal statistical
    error of <P>, the algorithm and its autocorrelations being the same): 32^4
    at beta = 6.0, same seed, FP64-18 / FP64-12 / FP32-18 / FP32-12.  Errors
    from 20 jackknife bins of nmeas / 20 sweeps, longer than tau_int."""
    import torch

    import paper_0904_0642_amd as su3hb
    from paper_0904_0642_amd.analysis import jackknife_mean, tau_int

    ext, beta = (32, 32, 32, 32), 6.0
    links = int(np.prod(ext)) * 4
    res = {"lattice": list(ext), "beta": beta, "thermalisation_sweeps": ntherm, "measured_sweeps": nmeas}
    for prec in (su3hb.FP64_18, su3hb.FP64_12, su3hb.FP32_18, su3hb.FP32_12):
        lat = su3hb.Lattice(ext, precision=prec, seed=11)
        lat.autotune(200)
        lat.sweep(beta, n_hit=n_hit, n_sweeps=ntherm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ser = lat.sweep_measure(beta, n_hit=n_hit, n_sweeps=nmeas)
        secs = time.perf_counter() - t0
        m, e = jackknife_mean(ser[:, 0], 20)
        tau, dtau, _ = tau_int(ser[:, 0])
        res[PREC_NAME[prec]] = {"rate": round(nmeas * links / secs, 1), "plaquette": m, "error": e,
                                "tau_int_sweeps": [round(tau, 1), round(dtau, 1)],
                                "spacelike": list(jackknife_mean(ser[:, 1], 20)),
                                "timelike": list(jackknife_mean(ser[:, 2], 20))}
        lat.close()
        torch.cuda.empty_cache()
    ref = res["fp64-18"]
    for k in ("fp64-12", "fp32-18", "fp32-12"):
        r = res[k]
        r["speedup_vs_fp64_at_equal_error"] = round(r["rate"] / ref["rate"], 3)
        r["delta_vs_fp64_in_sigma"] = round((r["plaquette"] - ref["plaquette"]) / np.hypot(r["error"], ref["error"]), 2)
        for obs in ("spacelike", "timelike"):
            (m, e), (m0, e0) = r[obs], ref[obs]
            r[obs + "_delta_vs_fp64_in_sigma"] = round((m - m0) / np.hypot(e, e0), 2)
    return res


def small_configs_leg(n_hit: int):
    """The paper's small runs at their full sweep counts on the GPU (FP64-18,
    plaquettes after every sweep, seed 1, the library's default launch).
    These lattices sit in the Infinity Cache, so only the rate is given."""
    import torch

    import paper_0904_0642_amd as su3hb

    out = {}
    for name, (ext, nlat, mask, cold, beta, sweeps) in SMALL_CONFIGS.items():
        lat = su3hb.Lattice(ext, nlat=nlat, dlt_mask=mask, precision=su3hb.FP64_18,
                            start=su3hb.COLD if cold else su3hb.HOT, seed=1)
        links = nlat * int(np.prod(ext)) * len(ext)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ser = lat.sweep_measure(beta, n_hit=n_hit, n_sweeps=sweeps)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        out[name] = {"value": round(sweeps * links / secs, 1), "unit": "link updates/s", "sweeps": sweeps,
                     "seconds": round(secs, 4), "beta": beta, "plaquette_last": float(ser[-1, 0])}
        lat.close()
    torch.cuda.empty_cache()
    return out


def oracle_small_configs(n_hit: int, threads: int):
    """The FP64 oracle on the same small runs, a sweep and a plaquette
    measurement at a time: config 1 in full, the others on a bounded sample
    of their sweeps (at least one, until about 2 s have passed), on all host
    threads and on one."""
    import oracle

    out = {}
    for name, (ext, nlat, mask, cold, beta, sweeps) in SMALL_CONFIGS.items():
        links = nlat * int(np.prod(ext)) * len(ext)
        res = {"unit": "link updates/s", "sweeps_in_full_run": sweeps}
        for label, th, budget in (("all_threads", threads, 2.0), ("single_thread", 1, 2.0)):
            o = oracle.Lattice(list(ext), nlat=nlat, dlt_mask=mask, seed=1, threads=th)
            if cold:
                o.cold_start()
            else:
                o.hot_start()
            done_sweeps, t0 = 0, time.perf_counter()
            while done_sweeps < sweeps:
                o.sweep(beta, nhit=n_hit)
                o.plaquette(beta)
                done_sweeps += 1
                if time.perf_counter() - t0 >= budget:
                    break
            secs = time.perf_counter() - t0
            rate = done_sweeps * links / secs
            res[label] = {"value": round(rate, 1), "cores": th, "sweeps_timed": done_sweeps,
                          "seconds": round(secs, 3),
                          "full_run_seconds": round(sweeps * links / rate, 2)}
            del o
        out[name] = res
    return out


def oracle_rate(name: str, n_hit: int, threads: int, min_secs: float, max_sweeps: int):
    """Link updates per second of the FP64 oracle on checkerboard slices of
    the hot-started lattice in sweep order (parity 0, 1; directions
    0..D-1), with OpenMP over the sites of a slice, until min_secs have
    passed or max_sweeps sweeps are done (at least one slice)."""
    import oracle

    ext, prec, beta = WORKLOADS[name]
    D = len(ext)
    o = oracle.Lattice(list(ext), seed=1, threads=threads)
    o.hot_start()
    V = int(np.prod(ext))
    slices = 0
    t0 = time.perf_counter()
    while slices < 2 * D * max_sweeps:
        o.update_slice(slices // D % 2, slices % D, beta, beta, nhit=n_hit)
        slices += 1
        if time.perf_counter() - t0 >= min_secs:
            break
    secs = time.perf_counter() - t0
    n = slices * (V // 2)
    del o
    return n / secs, slices, n, secs


def cpu_baseline(name: str, n_hit: int, min_secs: float = 10.0, max_sweeps: int = 6):
    """The FP64 oracle on a bounded sample of the same workload, on all host
    threads the run may use and on one thread, and on the paper's small runs
    (oracle_small_configs)."""
    ext, prec, beta = WORKLOADS[name]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rate, slices, n, secs = oracle_rate(name, n_hit, threads, min_secs, max_sweeps)
    rate1, slices1, n1, secs1 = oracle_rate(name, n_hit, 1, min_secs / 2, max_sweeps)
    return {"value": rate, "unit": "link updates/s", "cores": threads, "kind": "oracle",
            "host_cpus": os.cpu_count(),
            "sample": f"{slices} checkerboard slices in sweep order ({n} link updates) of the hot-started "
                      f"{'x'.join(map(str, ext))} lattice at beta={beta}, n_hit={n_hit}, FP64 C oracle, "
                      f"OpenMP {threads} threads, {secs:.2f} s",
            "single_thread": {"value": rate1, "unit": "link updates/s", "cores": 1,
                              "sample": f"{slices1} slices ({n1} link updates), 1 thread, {secs1:.2f} s"},
            "small_configs": oracle_small_configs(n_hit, threads)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed sweeps")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="48^4-fp64", choices=sorted(WORKLOADS))
    ap.add_argument("--compare", default="64^4-fp32-12", help="second leg ('' to skip)")
    ap.add_argument("--n-hit", type=int, default=8)
    ap.add_argument("--autotune-ms", type=int, default=1600)
    ap.add_argument("--launch", default="", help="block,order,waves for the main leg instead of autotuning")
    ap.add_argument("--compare-launch", default="", help="block,order,waves for the comparison leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-legs", action="store_true", help="skip the batch, DLT and precision legs")
    ap.add_argument("--extra-legs", default=",".join(EXTRA_LEGS),
                    help="comma-separated subset of the extra legs to run: " + ", ".join(EXTRA_LEGS))
    ap.add_argument("--batch-launch", default="", help="block,order,waves for the batch leg instead of autotuning")
    ap.add_argument("--batch-modes", default="graph_per_slice,persistent",
                    help="batch modes to time: graph_per_slice, persistent (cooperative launch)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MiB (for scaling HBM counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the whole lattice is resident on a single MI355X; "
              "runs on more than one GPU are not supported (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    import paper_0904_0642_amd as su3hb
    su3hb.lib()

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()

    def done(what):
        # one progress line per finished leg, on stderr (stdout carries the JSON line)
        print(f"[bench] {what} done", file=sys.stderr, flush=True)

    main_leg = run_leg(args.workload, args.steps, args.warmup, args.n_hit, args.autotune_ms,
                       parse_launch(args.launch))
    done(args.workload)
    legs = {}
    if args.compare and args.compare != args.workload:
        legs[args.compare] = run_leg(args.compare, args.steps, args.warmup, args.n_hit, args.autotune_ms,
                                     parse_launch(args.compare_launch))
        done(args.compare)

    ext, prec, beta = WORKLOADS[args.workload]
    line = {
        "metric": "SU(3) link updates/sec + % HBM roofline, FP32 vs FP64 at equal <P> error",
        "value": round(main_leg["rate"], 1),
        "unit": "link updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_leg["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": PREC_DTYPE[prec],
        "data": "synthetic (Haar start from the seeded Philox stream)",
        "config": {"workload": f"checkerboard CM/FHKP heatbath, D=4 {'x'.join(map(str, ext))} periodic torus, "
                               f"beta={beta}, {PREC_NAME[prec]} links, hot start seed 1, n_hit={args.n_hit}, "
                               f"plaquette every sweep",
                   "lattice": list(ext), "precision": PREC_NAME[prec], "beta": beta, "n_hit": args.n_hit,
                   "links_per_sweep": main_leg["links_per_sweep"], "launch": main_leg["launch"]},
        "roofline": main_leg["roofline"],
        "update_kernel_ms": round(main_leg["update_kernel_ms"], 5),
        "plaquette_kernel_ms": round(main_leg["plaquette_kernel_ms"], 5),
        "plaquette_first_last": main_leg["plaquette_first_last"],
    }
    for name, leg in legs.items():
        line["compare_" + name] = {
            "value": round(leg["rate"], 1), "unit": "link updates/s", "ms_per_step": round(leg["ms_per_step"], 4),
            "roofline": leg["roofline"], "update_kernel_ms": round(leg["update_kernel_ms"], 5),
            "plaquette_kernel_ms": round(leg["plaquette_kernel_ms"], 5), "launch": leg["launch"],
            "plaquette_first_last": leg["plaquette_first_last"],
            "rate_ratio_vs_main": round(leg["rate"] / main_leg["rate"], 3),
        }
    extra = set() if args.no_extra_legs else {x for x in args.extra_legs.split(",") if x}
    unknown = extra - set(EXTRA_LEGS)
    if unknown:
        print(f"unknown extra legs: {sorted(unknown)}", file=sys.stderr)
        sys.exit(2)
    if "batch" in extra:
        line["batch_128_replicas"] = batch_leg(args.steps, args.warmup, args.n_hit, args.autotune_ms,
                                               launch=parse_launch(args.batch_launch),
                                               modes=tuple(args.batch_modes.split(",")))
        done("batch")
    if "dlt" in extra:
        line["dlt_2x24^3x8"] = dlt_leg(args.n_hit, args.autotune_ms)
        done("double-layered torus")
    if "precision" in extra:
        line["precision_study"] = precision_study(args.n_hit)
        done("precision study")
    if "overrelax" in extra:
        line["overrelaxation_" + args.workload] = overrelax_leg(args.workload, args.steps, args.warmup,
                                                                args.autotune_ms)
        done("overrelaxation")
    if "full_size" in extra:
        for name in ("64^4-fp32-18", "48^4-fp64-12"):
            if name in (args.workload, args.compare):
                continue
            leg = run_leg(name, args.steps, args.warmup, args.n_hit, args.autotune_ms)
            done(name)
            line["full_size_" + name] = {
                "value": round(leg["rate"], 1), "unit": "link updates/s",
                "ms_per_step": round(leg["ms_per_step"], 4), "roofline": leg["roofline"],
                "update_kernel_ms": round(leg["update_kernel_ms"], 5), "launch": leg["launch"],
                "rate_ratio_vs_main": round(leg["rate"] / main_leg["rate"], 3),
            }
    if "small_configs" in extra:
        line["small_configs"] = small_configs_leg(args.n_hit)
        done("small configs")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.n_hit)
        done("cpu baseline")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
