"""Error analysis of Monte Carlo time series, in the form the paper uses
(Sec. 3.2-3.4): binned jackknife error bars, the Gaussian difference test and
the integrated autocorrelation time.  Host-side numpy; it analyses measured
series and holds none of the update's arithmetic.
"""
from __future__ import annotations

import math

import numpy as np


def jackknife_mean(series, nbins: int = 32):
    """Mean and binned-jackknife error bar of a time series (the first
    nbins * floor(N / nbins) entries, split into nbins consecutive bins)."""
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
    """Gaussian difference test: the probability that two estimates with
    Gaussian errors e1, e2 of one quantity differ by at least |m1 - m2|."""
    d = abs(m1 - m2) / math.sqrt(e1 * e1 + e2 * e2)
    return math.erfc(d / math.sqrt(2.0))


def autocorrelation(series, tmax: int) -> np.ndarray:
    """Normalised autocorrelation rho(t), t = 0..tmax, via FFT."""
    x = np.asarray(series, dtype=np.float64)
    x = x - x.mean()
    n = len(x)
    f = np.fft.rfft(x, 2 * n)
    c = np.fft.irfft(f * np.conj(f))[: tmax + 1] / np.arange(n, n - tmax - 1, -1)
    return c / c[0]


def tau_int(series, c: float = 6.0):
    """Integrated autocorrelation time tau_int = 1 + 2 sum_{t>=1} rho(t) in
    units of the series spacing, summed up to the first window W with
    W >= c tau_int(W) (automatic windowing), and its statistical error
    tau_int sqrt(2 (2W + 1) / N).  With this normalisation the error of the
    mean is sqrt(tau_int var / N).  Returns (tau_int, error, W)."""
    x = np.asarray(series, dtype=np.float64)
    n = len(x)
    rho = autocorrelation(x, max(1, n // 4))
    tau = 1.0
    for w in range(1, len(rho)):
        tau += 2.0 * rho[w]
        if w >= c * tau:
            return tau, tau * math.sqrt(2.0 * (2 * w + 1) / n), w
    return tau, tau * math.sqrt(2.0 * (2 * (len(rho) - 1) + 1) / n), len(rho) - 1
