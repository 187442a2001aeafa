"""Pins for the oracle's phi_k functions (Section 2.2 definition)."""
from math import factorial

import mpmath
import numpy as np
import pytest

from oracle.phi import phi

ZS = [-1e6, -1e3, -50.0, -3.0, -1.0000001, -1.0, -0.999, -0.5, -1e-3, -1e-9, 0.0,
      1e-7, 0.3, 1.0, 1.5, 4.0]


def _mp_phi(k, z):
    """phi_k by 40-digit quadrature of the integral definition (k >= 1)."""
    mpmath.mp.dps = 40
    z = mpmath.mpf(z)
    if k == 0:
        return mpmath.e ** z
    f = lambda th: mpmath.e ** ((1 - th) * z) * th ** (k - 1) / mpmath.factorial(k - 1)
    # split near theta = 1 where the integrand concentrates for large -z
    pts = [0, 1]
    if z < -10:
        pts = [0, 1 - 50 / abs(z), 1 - 10 / abs(z), 1] if abs(z) > 50 else [0, 0.5, 1]
    return mpmath.quad(f, pts)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_phi_matches_integral_definition(k):
    for z in ZS:
        ref = float(_mp_phi(k, z))
        got = float(phi(k, z))
        assert got == pytest.approx(ref, rel=3e-15, abs=0), (k, z)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_phi_at_zero(k):
    assert float(phi(k, 0.0)) == pytest.approx(1.0 / factorial(k), rel=1e-16)


def test_phi_recursion_where_well_conditioned():
    z = np.array([-40.0, -7.0, -2.0, 2.0, 9.0])
    for k in range(3):
        np.testing.assert_allclose(phi(k + 1, z), (phi(k, z) - 1.0 / factorial(k)) / z, rtol=1e-14)


def test_phi_vectorised_and_no_nan_for_huge_arguments():
    z = -np.logspace(-12, 12, 200)
    for k in range(3):
        v = phi(k, z)
        assert np.all(np.isfinite(v))
    np.testing.assert_allclose(phi(1, np.array([-1e12])), [1e-12], rtol=1e-12)
    np.testing.assert_allclose(phi(2, np.array([-1e12])), [1e-12], rtol=1e-11)
