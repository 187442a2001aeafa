"""Pins for the oracle's finite element matrices and their diagonalisation.

Section 4 states A = (h/6) R and B = (1/h) G^D, the sine eigenvectors and the
1D eigenvalues; the Q1 matrices are also rebuilt by element quadrature.
"""
import numpy as np
import pytest
import scipy.fft
import scipy.linalg

from oracle import fem, spectral


@pytest.mark.parametrize("N,h", [(2, 0.5), (5, 0.2), (16, 1.0 / 16), (9, 0.37)])
def test_1d_matrices_match_section4_tridiagonal_forms(N, h):
    A, B = fem.assemble_1d(N, h)
    n = N - 1
    R = 4.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    G = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    np.testing.assert_allclose(A, h / 6.0 * R, rtol=0, atol=1e-15)
    np.testing.assert_allclose(B, G / h, rtol=0, atol=1e-12)


@pytest.mark.parametrize("N,h,D", [
    ([5], [0.3], 1.3),
    ([4, 3], [0.25, 0.4], 0.7),
    ([3, 4, 3], [0.5, 0.2, 0.3], 2.0),
])
def test_kronecker_assembly_equals_q1_element_quadrature(N, h, D):
    M, K = fem.mass_stiffness(N, h, D)
    Mq, Kq = fem.q1_quadrature_assembly(N, h, D)
    np.testing.assert_allclose(M.toarray(), Mq, rtol=0, atol=1e-15)
    np.testing.assert_allclose(K.toarray(), Kq, rtol=0, atol=1e-13)


@pytest.mark.parametrize("N,h", [(4, 0.25), (16, 1.0 / 16), (64, 1.0 / 64), (37, 0.11)])
def test_1d_eigenvalues_closed_form(N, h):
    A, B = fem.assemble_1d(N, h)
    mu = scipy.linalg.eigh(B, A, eigvals_only=True)
    k = np.arange(1, N)
    c = np.cos(k * np.pi / N)
    closed = 6.0 * (1.0 - c) / (h * h * (2.0 + c))
    # generalised eigh is backward stable; 1e-12 covers its forward error at N = 64
    np.testing.assert_allclose(np.sort(mu), np.sort(closed), rtol=1e-12)


def test_printed_mass_eigenvalue_needs_the_square_and_P_needs_scaling():
    """Section 4's lambda^A prints sin where sin^2 is meant; P^2 = (N/2) I."""
    N, h = 16, 1.0 / 16
    n = N - 1
    A, B = fem.assemble_1d(N, h)
    i = np.arange(1, N)
    P = np.sin(np.outer(i, i) * np.pi / N)
    np.testing.assert_allclose(P @ P, (N / 2.0) * np.eye(n), atol=1e-12)
    S = np.sqrt(2.0 / N) * P
    printed = (h / 6.0) * (6.0 - 4.0 * np.sin(i * np.pi / (2 * N)))
    squared = (h / 6.0) * (6.0 - 4.0 * np.sin(i * np.pi / (2 * N)) ** 2)
    np.testing.assert_allclose(S @ A @ S, np.diag(squared), atol=1e-15)
    assert np.max(np.abs(S @ A @ S - np.diag(printed))) > 1e-3
    lamB = (4.0 / h) * np.sin(i * np.pi / (2 * N)) ** 2
    np.testing.assert_allclose(S @ B @ S, np.diag(lamB), atol=1e-12)
    # the printed orthogonal decomposition with unscaled P fails
    assert np.max(np.abs(P @ np.diag(squared) @ P.T - A)) > 1e-2


@pytest.mark.parametrize("N", [2, 3, 8, 33])
def test_sine_eigenvectors_and_library_dst(N):
    h = 1.0 / N
    A, B = fem.assemble_1d(N, h)
    mu, V = scipy.linalg.eigh(B, A)
    i = np.arange(1, N)
    S = np.sqrt(2.0 / N) * np.sin(np.outer(i, i) * np.pi / N)
    np.testing.assert_allclose(S @ S, np.eye(N - 1), atol=1e-14)
    # eigh sorts ascending; mode k has eigenvector proportional to sin(j k pi / N)
    for k in range(N - 1):
        v = V[:, k] / np.linalg.norm(V[:, k])
        s = S[:, k]
        assert abs(abs(float(v @ s)) - 1.0) < 1e-12
    x = np.random.default_rng(0).standard_normal(N - 1)
    np.testing.assert_allclose(scipy.fft.dst(x, type=1, norm="ortho"), S @ x, atol=1e-14)


def test_sine_eigs_match_generalised_problem():
    for N, h in [(7, 0.3), (50, 0.02)]:
        lamA, lamB = spectral.sine_eigs(N, h)
        A, B = fem.assemble_1d(N, h)
        mu = scipy.linalg.eigh(B, A, eigvals_only=True)
        np.testing.assert_allclose(np.sort(lamB / lamA), mu, rtol=1e-12)


def test_node_coords_and_mesh_layout():
    xs = fem.node_coords([4, 3], [0.5, 1.0 / 3], origin=[1.0, -1.0])
    np.testing.assert_allclose(xs[0], [1.5, 2.0, 2.5])
    np.testing.assert_allclose(xs[1], [-1.0 + 1.0 / 3, -1.0 + 2.0 / 3])
    X = fem.mesh([4, 3], [0.5, 1.0 / 3], origin=[1.0, -1.0])
    assert X[0].shape == (1, 3) and X[1].shape == (2, 1)
