"""Pins for the oracle's energy and quadrature error norms (oracle.norms).

* allen_cahn_energy: the gradient term (D/2) U^T K_1 U against the closed-form
  eigenvalues of Section 4 on a sine-product state and against an element
  quadrature of |grad u_h|^2; the potential term against the exact integral
  of the double-well potential for a state the nodal (trapezoid) rule
  integrates exactly.
* quadrature_errors (any d): equal to the 2D routine on 2D data, zero for a
  multilinear solution (Q1 reproduces it), and the exact integrals of a sine
  product and its gradient.
"""
import numpy as np
import pytest

from oracle import fem, norms, problems


def _lam_A(k, N, h):
    """Mass eigenvalue of the 1D interior matrix (Section 4, with the square restored)."""
    return h / 6.0 * (4.0 + 2.0 * np.cos(k * np.pi / N))


def _lam_B(k, N, h):
    """Stiffness eigenvalue of the 1D interior matrix (Section 4)."""
    return 2.0 / h * (1.0 - np.cos(k * np.pi / N))


def _sine_state(N, h, modes):
    X = fem.mesh(N, h)
    U = 1.0
    for a, x in enumerate(X):
        U = U * np.sin(modes[a] * np.pi * x / (N[a] * h[a]))
    return U


@pytest.mark.parametrize("N,h,modes", [([12], [1 / 12], [3]), ([10, 7], [0.1, 0.13], [2, 5]),
                                       ([6, 8, 5], [1 / 6, 0.125, 0.21], [1, 3, 4])])
def test_gradient_term_of_sine_mode_from_section4_eigenvalues(N, h, modes):
    """U = prod_a sin(k_a pi x_a / L_a): U^T K_1 U = sum_a lam^B_{k_a} prod_{b != a} lam^A_{k_b}
    times prod_a N_a / 2 (the squared norm of each discrete sine vector)."""
    D = 0.7
    U = _sine_state(N, h, modes)
    d = len(N)
    closed = 0.0
    for a in range(d):
        term = _lam_B(modes[a], N[a], h[a])
        for b in range(d):
            if b != a:
                term *= _lam_A(modes[b], N[b], h[b])
        closed += term
    closed *= np.prod([n / 2.0 for n in N])
    grad = norms.allen_cahn_energy(N, h, D, U) - norms.allen_cahn_energy(N, h, 0.0, U)
    np.testing.assert_allclose(grad, 0.5 * D * closed, rtol=1e-12)


@pytest.mark.parametrize("N,h", [([9, 6], [1 / 9, 1 / 6]), ([4, 5, 3], [0.25, 0.2, 1 / 3])])
def test_gradient_term_equals_element_quadrature(N, h):
    """(D/2) U^T K_1 U = (D/2) int |grad u_h|^2, the integral taken by Gauss points of the
    Q1 function (quadrature_errors with a zero exact solution gives H1^2 - L2^2)."""
    D = 1.3
    U = np.random.default_rng(4).uniform(-1.0, 1.0, tuple(n - 1 for n in reversed(N)))
    zero = lambda t, X: 0.0 * X[0]
    zgrad = lambda t, X: [0.0 * X[0] for _ in X]
    l2, h1 = norms.quadrature_errors(N, h, None, U, zero, zgrad, 0.0)
    grad = norms.allen_cahn_energy(N, h, D, U) - norms.allen_cahn_energy(N, h, 0.0, U)
    np.testing.assert_allclose(grad, 0.5 * D * (h1 ** 2 - l2 ** 2), rtol=1e-12)


@pytest.mark.parametrize("d,N", [(1, 9), (2, 16), (3, 8)])
def test_potential_term_exact_integral(d, N):
    """D = 0 leaves prod(h) sum_i (U_i^2 - 1)^2 / 4 over interior nodes.  For
    u = prod_a sin(pi x_a) on the unit cube the nodal rule over all nodes is the
    trapezoid rule, exact for these trigonometric polynomials, so the interior sum
    is int (u^2 - 1)^2 / 4 minus the boundary nodes' weight times (0 - 1)^2 / 4."""
    Ns, h = [N] * d, [1.0 / N] * d
    U = _sine_state(Ns, h, [1] * d)
    exact = 0.25 * ((3.0 / 8.0) ** d - 2.0 * 0.5 ** d + 1.0)
    boundary_weight = 1.0 - ((N - 1) / N) ** d
    np.testing.assert_allclose(norms.allen_cahn_energy(Ns, h, 0.0, U),
                               exact - 0.25 * boundary_weight, rtol=1e-13)


def test_energy_of_constant_states():
    N, h = [7, 5], [1 / 7, 0.2]
    n = 6 * 4
    # zero state: potential 1/4 per node, no gradient
    np.testing.assert_allclose(norms.allen_cahn_energy(N, h, 0.9, np.zeros((4, 6))),
                               np.prod(h) * n / 4.0, rtol=1e-14)
    # unit state: no potential; gradient of the function that is 1 inside, 0 on the boundary:
    # per axis 1^T B 1 = 2/h and 1^T A 1 = h (N - 4/3) from the tridiagonal forms
    one = (2.0 / h[0]) * h[1] * (N[1] - 4.0 / 3.0) + (2.0 / h[1]) * h[0] * (N[0] - 4.0 / 3.0)
    np.testing.assert_allclose(norms.allen_cahn_energy(N, h, 0.9, np.ones((4, 6))), 0.45 * one, rtol=1e-13)


def test_energy_slips_are_caught():
    """The closed forms above reject a halved diffusion coefficient and a dropped 1/4."""
    N, h = [10, 7], [0.1, 0.13]
    U = _sine_state(N, h, [2, 5])
    D = 0.7
    grad = norms.allen_cahn_energy(N, h, D, U) - norms.allen_cahn_energy(N, h, 0.0, U)
    wrong = norms.allen_cahn_energy(N, h, D / 2, U) - norms.allen_cahn_energy(N, h, 0.0, U)
    assert abs(wrong / grad - 0.5) < 1e-12
    pot = norms.allen_cahn_energy(N, h, 0.0, np.zeros((6, 9)))
    assert abs(pot - np.prod(h) * 54) > 0.5 * pot


@pytest.mark.parametrize("N,h", [([12, 9], [1 / 12, 1 / 9]), ([7, 16], [1 / 7, 1 / 16])])
def test_quadrature_errors_equal_2d_routine(N, h):
    """The any-d routine equals the 2D one where the exact solution vanishes on the
    boundary (both then use zero boundary values)."""
    U = np.random.default_rng(8).uniform(-1.0, 1.0, (N[1] - 1, N[0] - 1))
    ex = lambda t, X: problems.mms_u2_exact(t, X)

    def gr(t, X):
        x, y = X
        e = np.exp(-t)
        return [e * np.pi * np.cos(np.pi * x) * np.sin(np.pi * y),
                e * np.pi * np.sin(np.pi * x) * np.cos(np.pi * y)]

    a = norms.quadrature_errors(N, h, None, U, ex, gr, 0.3)
    b = norms.quadrature_errors_2d(N, h, (0.0, 0.0), U, ex, gr, 0.3)
    np.testing.assert_allclose(a, b, rtol=1e-13)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_quadrature_errors_of_sine_product(d):
    """U = 0, exact = prod_a sin(pi x_a) on the unit cube: L2^2 = 2^-d and
    H1^2 = 2^-d (1 + d pi^2), up to the Gauss rule's error on 12 elements per axis."""
    N, h = [12] * d, [1.0 / 12] * d
    U = np.zeros(tuple([11] * d))
    ex = lambda t, X: problems.mms_u2_exact(t, X)

    def gr(t, X):
        out = []
        for a in range(d):
            g = np.pi * np.cos(np.pi * X[a])
            for b in range(d):
                if b != a:
                    g = g * np.sin(np.pi * X[b])
            out.append(g)
        return out

    l2, h1 = norms.quadrature_errors(N, h, None, U, ex, gr, 0.0)
    np.testing.assert_allclose(l2 ** 2, 0.5 ** d, rtol=1e-9)
    np.testing.assert_allclose(h1 ** 2, 0.5 ** d * (1.0 + d * np.pi ** 2), rtol=1e-9)


@pytest.mark.parametrize("N", [[5], [4, 6], [3, 4, 5]])
def test_quadrature_errors_vanish_for_multilinear_solution(N):
    """Q1 reproduces prod_a (1 + c_a x_a): with its nodal values the errors are rounding."""
    d = len(N)
    h = [0.3, 0.2, 0.25][:d]
    c = [0.7, -1.1, 2.0][:d]
    def ex(t, X):
        v = 1.0
        for a in range(d):
            v = v * (1.0 + c[a] * X[a])
        return v

    def gr(t, X):
        out = []
        for a in range(d):
            g = c[a] + 0.0 * X[a]
            for b in range(d):
                if b != a:
                    g = g * (1.0 + c[b] * X[b])
            out.append(g)
        return out

    U = ex(0.0, fem.mesh(N, h))
    l2, h1 = norms.quadrature_errors(N, h, None, U, ex, gr, 0.0)
    assert l2 < 1e-14 and h1 < 1e-13
