"""Analysis tooling for Monte Carlo time series: binned jackknife and the
Gaussian difference test (the error analysis the paper uses, Sec. 3.2-3.4)."""
from __future__ import annotations

import math

import numpy as np


def jackknife_mean(series, nbins: int = 32):
    """Mean and binned-jackknife error bar of a time series."""
    x = np.asarray(series, dtype=np.float64)
    n = (len(x) // nbins) * nbins
    if n < nbins:
        raise ValueError("series shorter than the number of bins")
    bins = x[:n].reshape(nbins, -1).mean(axis=1)
    total = bins.sum()
    jk = (total - bins) / (nbins - 1)
    mean = jk.mean()
    err = math.sqrt((nbins - 1) / nbins * np.sum((jk - mean) ** 2))
    return float(x[:n].mean()), err


def gaussian_difference_q(m1, e1, m2, e2) -> float:
    """Q = probability that two Gaussian estimates differ by at least |m1-m2|."""
    d = abs(m1 - m2) / math.sqrt(e1 * e1 + e2 * e2)
    return math.erfc(d / math.sqrt(2.0))
