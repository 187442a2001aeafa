"""The functions phi_k of exponential Runge-Kutta methods (oracle; test infrastructure only).

Section 2.2 defines, for k >= 1,
    phi_k(z) = int_0^1 exp((1 - theta) z) theta^(k-1) / (k-1)! d theta,
with phi_0(z) = exp(z) and the recursion phi_{k+1}(z) = (phi_k(z) - phi_k(0)) / z.
The paper prints the recursion for k > 0; it holds for k >= 0 as well, with
phi_k(0) = 1/k!.

Expanding the exponential under the integral and using the Beta integral
int_0^1 (1-theta)^m theta^(k-1) d theta = m! (k-1)! / (m+k)! gives the series
    phi_k(z) = sum_{m >= 0} z^m / (m + k)!,
which this module uses for |z| <= 1.  For |z| > 1 it uses the recursion,
which then suffers no cancellation for the k <= 2 needed by EIFE1/EIFE2.
"""
from math import factorial

import numpy as np

_SERIES_TERMS = 30  # 1/30! < 4e-33: far below double rounding for |z| <= 1


def _series(k, z):
    out = np.zeros_like(z)
    for m in reversed(range(_SERIES_TERMS)):
        out = out * z + 1.0 / factorial(m + k)
    return out


def phi(k, z):
    """phi_k(z) in float64 for a scalar or array z (any sign)."""
    z = np.asarray(z, dtype=np.float64)
    scalar = z.ndim == 0
    z = np.atleast_1d(z)
    small = np.abs(z) <= 1.0
    out = np.empty_like(z)
    if np.any(small):
        out[small] = _series(k, z[small])
    big = ~small
    if np.any(big):
        zb = z[big]
        val = np.exp(zb)
        for j in range(k):
            val = (val - 1.0 / factorial(j)) / zb
        out[big] = val
    return out[0] if scalar else out
