"""Pins for the general s-stage exponential Runge-Kutta step of eq. (2.2)
(oracle/erk.py): the consistency conditions the paper states (eq. (2.3)), the
reduction to the independently written EIFE1/EIFE2 steps (eqs. (2.13),
(2.14)), exactness for forcing polynomial in t of degree < s against the
matrix exponential of an augmented system, and the observed order."""
import numpy as np
import pytest
import scipy.linalg

from oracle import erk, fem, norms, problems, spectral, stepper
from oracle.phi import phi

Z = -np.concatenate([np.linspace(0.0, 2.0, 21)[1:], np.geomspace(2.0, 5e4, 30)])


@pytest.mark.parametrize("nodes", [[0.0, 0.5], [0.0, 1 / 3, 2 / 3], [0.0, 0.5, 1.0], [0.0, 0.2, 0.7, 0.9]])
def test_consistency_conditions(nodes):
    chi_i, a, b, chi = erk.weights(nodes, Z)
    np.testing.assert_allclose(sum(b), phi(1, Z), rtol=1e-12, atol=1e-15)
    for i in range(1, len(nodes)):
        np.testing.assert_allclose(sum(a[i, j] for j in range(i)), nodes[i] * phi(1, nodes[i] * Z),
                                   rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(chi_i[i], np.exp(nodes[i] * Z), rtol=1e-15)
    np.testing.assert_allclose(chi, np.exp(Z), rtol=1e-15)


def test_full_node_reading_of_a_ij_breaks_consistency():
    """With the Lagrange polynomials of all nodes in a_ij the stated sum condition fails."""
    nodes = [0.0, 1 / 3, 2 / 3]
    z = -0.7
    i = 2
    full = [erk.lagrange_coefficients(nodes, j) for j in range(i)]
    from math import factorial
    a_full = [sum(al[k - 1] * nodes[i] ** k * factorial(k - 1) * phi(k, nodes[i] * z) for k in range(1, 4))
              for al in full]
    assert abs(sum(a_full) - nodes[i] * phi(1, nodes[i] * z)) > 1e-3


@pytest.mark.parametrize("s,c2", [(1, None), (2, 0.5), (2, 0.3)])
def test_reduces_to_eife1_and_eife2(s, c2):
    N, h = [9, 7], [1 / 9, 1 / 7]
    u0 = np.random.default_rng(s).uniform(-0.9, 0.9, (6, 8))
    b = spectral.make_basis("C", N, h, 0.02)
    nodes = [0.0] if s == 1 else [0.0, c2]
    got = erk.run(b, u0, problems.allen_cahn(), 0.07, 5, nodes)
    ref = stepper.run(b, u0, problems.allen_cahn(), 0.07, 5, s, c2=c2 or 0.5)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


def _augmented_poly(N, h, D, coef, T, u0):
    """Exact solution of M u' + K u = p(t) prod(h) 1, p(t) = sum_m coef[m] t^m, at time T."""
    M, K = fem.mass_stiffness(N, h, D)
    n = M.shape[0]
    L = np.linalg.solve(M.toarray(), K.toarray())
    v = np.linalg.solve(M.toarray(), np.full(n, float(np.prod(h))))
    deg = len(coef) - 1
    # state [u; y_0 .. y_deg] with y_m = t^m / m!: y_0' = 0, y_m' = y_{m-1}
    Zm = np.zeros((n + deg + 1, n + deg + 1))
    Zm[:n, :n] = -L
    from math import factorial
    for m in range(deg + 1):
        Zm[:n, n + m] = coef[m] * factorial(m) * v
        if m:
            Zm[n + m, n + m - 1] = 1.0
    y0 = np.concatenate([u0.reshape(-1), [1.0], np.zeros(deg)])
    return (scipy.linalg.expm(T * Zm) @ y0)[:n].reshape(u0.shape)


@pytest.mark.parametrize("nodes", [[0.0, 1 / 3, 2 / 3], [0.0, 0.5, 1.0]])
def test_three_stages_exact_for_quadratic_forcing(nodes):
    N, h, D = [6, 5, 4], [1 / 6, 1 / 5, 1 / 4], 0.5
    coef = [0.3, -1.1, 2.4]
    f = lambda t, X, U: np.full_like(U, coef[0] + coef[1] * t + coef[2] * t * t)
    u0 = np.random.default_rng(8).uniform(-1, 1, (3, 4, 5))
    for tier in "ABC":
        b = spectral.make_basis(tier, N, h, D)
        got = erk.run(b, u0, f, 0.11, 6, nodes)
        np.testing.assert_allclose(got, _augmented_poly(N, h, D, coef, 0.66, u0), rtol=0, atol=1e-13)
    # two stages are not exact for it
    b = spectral.make_basis("C", N, h, D)
    two = stepper.run(b, u0, f, 0.11, 6, 2)
    assert np.max(np.abs(two - _augmented_poly(N, h, D, coef, 0.66, u0))) > 1e-6


@pytest.mark.parametrize("nodes,order", [([0.0, 1 / 3, 2 / 3], 3.0), ([0.0, 0.5, 1.0], 2.0)])
def test_three_stage_order(nodes, order):
    """Manufactured problem u_t = Lap u + u^2 + g (2D, 16^2 intervals), temporal error against a
    fine same-grid run: nodes (0, 1/3, 2/3) converge at order 3, nodes (0, 1/2, 1) at order 2
    (observed; the paper gives no order for s >= 3)."""
    N, h = [16, 16], [1 / 16, 1 / 16]
    b = spectral.make_basis("C", N, h, 1.0)
    f = problems.mms_u2(1.0)
    u0 = problems.mms_u2_exact(0.0, fem.mesh(N, h))
    ref = erk.run(b, u0, f, 1.0 / 4096, 4096, [0.0, 1 / 3, 2 / 3])
    errs = [norms.discrete_norms(N, h, erk.run(b, u0, f, 1.0 / 2 ** k, 2 ** k, nodes) - ref)[0] for k in (4, 5, 6)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.2), rates


def test_variable_steps_match_the_two_stage_stepper():
    N, h = [9, 7], [1 / 9, 1 / 7]
    u0 = np.random.default_rng(6).uniform(-0.9, 0.9, (6, 8))
    b = spectral.make_basis("C", N, h, 0.02)
    taus = np.random.default_rng(7).uniform(0.01, 0.1, 7)
    got = erk.run(b, u0, problems.affine_t(0.2, 0.7), taus, 7, [0.0, 0.4], t0=0.3)
    ref = stepper.run(b, u0, problems.affine_t(0.2, 0.7), taus, 7, 2, c2=0.4, t0=0.3)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)
