"""Pins of the error analysis (CPU): the paper's own Gaussian difference test,
and closed forms for independent and AR(1) series."""
import math

import numpy as np

from stats import gaussian_difference_q, jackknife_mean, tau_int


def test_q_of_the_papers_two_results():
    # Sec. 3.2: act = 0.53811(19) (MPI) against 0.53770(18) (single processor)
    # gives Q = 0.12 in the Gaussian difference test
    q = gaussian_difference_q(0.53811, 0.00019, 0.53770, 0.00018)
    assert round(q, 2) == 0.12
    assert gaussian_difference_q(1.0, 0.1, 1.0, 0.1) == 1.0


def test_jackknife_of_independent_data():
    rng = np.random.default_rng(1)
    x = rng.normal(0.3, 2.0, size=2 ** 16)
    m, e = jackknife_mean(x, 32)
    assert abs(m - x.mean()) < 1e-15
    assert abs(e / (2.0 / math.sqrt(len(x))) - 1.0) < 0.35   # 32 bins: ~13% relative spread


def test_tau_int_of_an_ar1_series():
    # x_t = phi x_{t-1} + noise: rho(t) = phi^t, tau_int = (1 + phi) / (1 - phi)
    rng = np.random.default_rng(2)
    for phi in (0.0, 0.5, 0.9):
        n = 2 ** 18
        e = rng.normal(size=n)
        x = np.empty(n)
        x[0] = e[0] / math.sqrt(1 - phi * phi)
        for t in range(1, n):
            x[t] = phi * x[t - 1] + e[t]
        tau, err, w = tau_int(x)
        exact = (1 + phi) / (1 - phi)
        assert abs(tau - exact) < 4 * err + 0.02 * exact, (phi, tau, err, exact)
        # the binned error of the mean follows from tau_int
        m, e_mean = jackknife_mean(x, 32)
        assert abs(e_mean / math.sqrt(exact * x.var() / n) - 1.0) < 0.4
