"""Seeded synthetic inputs and named workload presets.

This module holds no arithmetic of the heatbath itself: it only draws seeds,
couplings, replica tables and generic random SU(3) matrices (for gauge
transformations in tests) from numpy's seeded generators.  Both the GPU path
and the CPU oracle consume what it produces.

The workloads mirror the lattices the paper runs on (D = 4 periodic tori of
extents 4^4 .. 16^3 x 4 at beta around 5.5-5.7, ordered or disordered starts,
the double-layered torus of Sec. 2.2) and scale them to one MI355X.  Every
input is synthetic: a start configuration is the ordered start (all links 1)
or the disordered start (Haar links drawn from the seeded Philox stream).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FP64_18 = 0
FP32_18 = 1
FP32_12 = 2
FP64_12 = 3
PRECISION_NAMES = {FP64_18: "fp64-18", FP32_18: "fp32-18", FP32_12: "fp32-12", FP64_12: "fp64-12"}
COLD = 1
HOT = 2


@dataclass
class LatticeSpec:
    extents: tuple
    beta0: float
    beta1: float | None = None
    nlat: int = 1
    dlt_mask: int = 0
    lat2test: bool = False
    precision: int = FP64_18
    start: int = HOT
    seed: int = 1
    n_hit: int = 8
    sweeps: int = 1
    name: str = ""

    @property
    def nd(self) -> int:
        return len(self.extents)

    @property
    def volume(self) -> int:
        return int(np.prod(self.extents))

    @property
    def links_per_sweep(self) -> int:
        return self.nlat * self.volume * self.nd

    @property
    def b1(self) -> float:
        return self.beta0 if self.beta1 is None else self.beta1


def preset(name: str) -> LatticeSpec:
    """Named workloads (sizes, couplings, starts)."""
    p = {
        # D=4 4^4 torus, beta=6.0, ordered start, n_hit=8, 20 sweeps, FP64, seed 1
        "small-4^4": LatticeSpec((4, 4, 4, 4), 6.0, start=COLD, seed=1, n_hit=8, sweeps=20,
                                 name="4^4 beta=6.0 cold fp64"),
        # D=4 16^4 torus, disordered start, 200 sweeps (beta 5.7 and 6.0)
        "16^4-b5.7": LatticeSpec((16, 16, 16, 16), 5.7, start=HOT, seed=1, sweeps=200,
                                 name="16^4 beta=5.7 hot fp64"),
        "16^4-b6.0": LatticeSpec((16, 16, 16, 16), 6.0, start=HOT, seed=1, sweeps=200,
                                 name="16^4 beta=6.0 hot fp64"),
        # D=2 32^2 torus at beta=4 (exactly solvable plaquette)
        "2d-32^2": LatticeSpec((32, 32), 4.0, start=HOT, seed=1, sweeps=20000,
                               name="2D 32^2 beta=4.0 hot fp64"),
        # double-layered torus, 24^3 x 8 per layer, all directions glued
        "dlt-24^3x8": LatticeSpec((24, 24, 24, 8), 5.69, nlat=2, dlt_mask=0xF, precision=FP32_18,
                                  start=HOT, seed=1, sweeps=500,
                                  name="DLT 2x(24^3x8) beta=5.69 fp32"),
        # large single-lattice workloads sized for one GPU's HBM
        "48^4-fp64": LatticeSpec((48, 48, 48, 48), 6.2, precision=FP64_18, start=HOT, seed=1,
                                 sweeps=100, name="48^4 beta=6.2 fp64-18"),
        "64^4-fp32-12": LatticeSpec((64, 64, 64, 64), 6.2, precision=FP32_12, start=HOT, seed=1,
                                    sweeps=100, name="64^4 beta=6.2 fp32-12"),
        "64^4-fp32-18": LatticeSpec((64, 64, 64, 64), 6.2, precision=FP32_18, start=HOT, seed=1,
                                    sweeps=100, name="64^4 beta=6.2 fp32-18"),
    }
    return p[name]


@dataclass
class ReplicaTable:
    extents: list = field(default_factory=list)   # per replica, tuple of D extents
    betas: list = field(default_factory=list)
    seeds: list = field(default_factory=list)
    starts: list = field(default_factory=list)

    def __len__(self) -> int:
        return len(self.extents)

    @property
    def links_per_sweep(self) -> int:
        return int(sum(len(e) * int(np.prod(e)) for e in self.extents))


def replica_table(n: int = 128, seed: int = 7, shapes=((8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 4)),
                  beta_lo: float = 5.5, beta_hi: float = 6.5, start: int = HOT) -> ReplicaTable:
    """n independent replicas: shapes round-robin, beta uniform in [beta_lo, beta_hi]."""
    rng = np.random.default_rng(seed)
    t = ReplicaTable()
    betas = rng.uniform(beta_lo, beta_hi, size=n)
    seeds = rng.integers(1, 2**63 - 1, size=n, dtype=np.int64)
    for r in range(n):
        t.extents.append(tuple(shapes[r % len(shapes)]))
        t.betas.append(float(betas[r]))
        t.seeds.append(int(seeds[r]))
        t.starts.append(start)
    return t


def random_su3(rng: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-random SU(3) matrices from QR of complex Gaussian matrices
    (generic linear algebra, independent of the heatbath's own start)."""
    z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q * np.exp(-1j * np.angle(det) / 3.0)[:, None, None]
    return q


def seeds(n: int, seed: int = 12345) -> list:
    rng = np.random.default_rng(seed)
    return [int(v) for v in rng.integers(1, 2**63 - 1, size=n, dtype=np.int64)]
