"""Closed forms used to pin the oracle (no code shared with either implementation).

* ``u_exact(beta)``: the SU(3) one-plaquette expectation <(1/3) Re Tr U> for
  the weight exp((beta/3) Re Tr U) under Haar measure.  The one-link integral
  z(beta) = sum_{q in Z} det[I_{q+i-j}(beta/3)]_{i,j=1..3} (Weyl integration
  formula for SU(N) with the Bessel-function character expansion), and
  u = d ln z / d beta.  In two dimensions every closed surface of large area
  has <P> = u(beta) up to corrections of order u^{N_p}; in four dimensions
  strong coupling gives <P> = u(beta) + O(u^5).
* ``kp_acceptance(alpha)``: probability that one Kennedy-Pendleton proposal is
  accepted, sqrt(2 pi alpha) exp(-alpha) I_1(alpha).
* ``x0_mean(alpha)``: <x0> under sqrt(1-x0^2) exp(alpha x0), I_2/I_1.
* ``x0_cdf(alpha)``: numerical CDF of that density.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, special


def _z_and_dz(beta: float, qmax: int = 40):
    x = beta / 3.0
    z = 0.0
    dz = 0.0
    for q in range(-qmax, qmax + 1):
        idx = np.array([[q + i - j for j in range(3)] for i in range(3)])
        # exponentially scaled Bessel functions: common factor exp(3x) drops out of u
        M = special.ive(idx, x)
        # dI_n(x)/dx = (I_{n-1} + I_{n+1})/2 and dx/dbeta = 1/3
        dM = (special.ive(idx - 1, x) + special.ive(idx + 1, x)) / 6.0
        z += np.linalg.det(M)
        for c in range(3):
            Mc = M.copy()
            Mc[:, c] = dM[:, c]
            dz += np.linalg.det(Mc)
    return z, dz


def u_exact(beta: float) -> float:
    if beta == 0.0:
        return 0.0
    # Every entry of M and of the derivative columns carries the same factor
    # exp(-x) from ive, so each determinant carries exp(-3x) and the ratio
    # dz/z equals d ln z_true / d beta exactly.
    z, dz = _z_and_dz(beta)
    return dz / z


def kp_acceptance(alpha: float) -> float:
    return float(np.sqrt(2.0 * np.pi * alpha) * special.ive(1, alpha))


def x0_mean(alpha: float) -> float:
    return float(special.ive(2, alpha) / special.ive(1, alpha))


def x0_cdf(alpha: float):
    """Return a callable CDF of the density ~ sqrt(1-x^2) exp(alpha (x-1)) on [-1,1]."""
    xs = np.linspace(-1.0, 1.0, 200001)
    pdf = np.sqrt(np.clip(1.0 - xs * xs, 0.0, None)) * np.exp(alpha * (xs - 1.0))
    cdf = integrate.cumulative_trapezoid(pdf, xs, initial=0.0)
    cdf /= cdf[-1]
    return lambda x: np.interp(x, xs, cdf)


def dlt_two_coupling_exact(n0, n1, beta0, beta1):
    """Exact 2D double-layered torus, both directions glued, two couplings.
    On a closed 2D surface every plaquette is an independent variable up to
    exponentially small global constraints, so <P_p> = u(beta_p).  A layer-0
    plaquette keeps all four links in layer 0 (tag rule: beta0) unless it
    touches the last row or column, whose forward neighbours sit in layer 1;
    every other plaquette carries beta1.  Returns the layer-0 and layer-1
    averages and the weighted sum sum_p beta_p <P_p>."""
    n = n0 * n1
    n_b0 = (n0 - 1) * (n1 - 1)
    u0, u1 = u_exact(beta0), u_exact(beta1)
    layer0 = (n_b0 * u0 + (n - n_b0) * u1) / n
    weighted = n_b0 * beta0 * u0 + (2 * n - n_b0) * beta1 * u1
    return layer0, u1, weighted
