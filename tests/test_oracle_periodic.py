"""Pins for the oracle's periodic boundary conditions (end of Section 4) and the
Flory-Huggins reaction of Example 5.3.

Section 4 states B = (1/h) G^P for the periodic case, but its printed sine
vectors are not a basis (one of them vanishes) and its printed eigenvalues,
with (i - 1) pi / (2N) arguments, are not the spectrum; the reading used here
is the real Fourier basis of the circulant matrices with
lambda^A = (h/6)(4 + 2 cos(2 pi k/N)), lambda^B = (2/h)(1 - cos(2 pi k/N)).
Each pin checks the oracle against something it does not compute itself:
the stated matrix forms, element quadrature, dense eigendecomposition, the
matrix exponential, or an invariant of the equation.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import fem, norms, problems, spectral, stepper


@pytest.mark.parametrize("N,h", [(3, 0.3), (4, 0.25), (7, 0.13), (16, 1.0 / 16)])
def test_periodic_1d_matrices_match_circulant_forms(N, h):
    A, B = fem.assemble_1d(N, h, "periodic")
    R = 4.0 * np.eye(N)
    G = 2.0 * np.eye(N)
    for j in range(N):
        R[j, (j + 1) % N] += 1.0
        R[j, (j - 1) % N] += 1.0
        G[j, (j + 1) % N] -= 1.0
        G[j, (j - 1) % N] -= 1.0
    np.testing.assert_allclose(A, h / 6.0 * R, rtol=0, atol=1e-15)
    np.testing.assert_allclose(B, G / h, rtol=0, atol=1e-12)


@pytest.mark.parametrize("N,h,D", [
    ([5], [0.3], 1.3),
    ([4, 3], [0.25, 0.4], 0.7),
    ([3, 4, 3], [0.5, 0.2, 0.3], 2.0),
])
def test_periodic_kronecker_assembly_equals_q1_element_quadrature(N, h, D):
    M, K = fem.mass_stiffness(N, h, D, "periodic")
    Mq, Kq = fem.q1_quadrature_assembly(N, h, D, bc="periodic")
    np.testing.assert_allclose(M.toarray(), Mq, rtol=0, atol=1e-15)
    np.testing.assert_allclose(K.toarray(), Kq, rtol=0, atol=1e-13)


@pytest.mark.parametrize("N,h", [(4, 0.25), (9, 0.11), (16, 1.0 / 16), (64, 1.0 / 64)])
def test_periodic_eigenvalues_closed_form(N, h):
    A, B = fem.assemble_1d(N, h, "periodic")
    mu = scipy.linalg.eigh(B, A, eigvals_only=True)
    lamA, lamB = spectral.fourier_eigs(N, h)
    np.testing.assert_allclose(np.sort(mu), np.sort(lamB / lamA), rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("N", [4, 5, 8, 9, 12])
def test_real_fourier_transform_diagonalises_the_periodic_matrices(N):
    """R (built from the library real FFT) is orthogonal and R A R^T, R B R^T are the
    closed-form diagonals, with A and B assembled from element matrices."""
    h = 1.0 / N
    R = spectral.real_fourier(np.eye(N), 0)  # column j = R e_j
    np.testing.assert_allclose(R @ R.T, np.eye(N), atol=1e-14)
    A, B = fem.assemble_1d(N, h, "periodic")
    lamA, lamB = spectral.fourier_eigs(N, h)
    np.testing.assert_allclose(R @ A @ R.T, np.diag(lamA), atol=1e-15)
    np.testing.assert_allclose(R @ B @ R.T, np.diag(lamB), atol=1e-12)
    # and the inverse is the transpose
    x = np.random.default_rng(N).standard_normal(N)
    np.testing.assert_allclose(spectral.real_fourier(R @ x, 0, inverse=True), x, atol=1e-14)


def test_printed_periodic_basis_and_eigenvalues_are_not_the_spectrum():
    """The printed vectors sin(ij pi/N), i, j = 1..N, are not a basis (column N vanishes),
    and the printed lambda^A_i = (h/6)(6 - 4 sin((i-1) pi/(2N))) is not the spectrum of A."""
    N, h = 8, 1.0 / 8
    A, _ = fem.assemble_1d(N, h, "periodic")
    i = np.arange(1, N + 1)
    P = np.sin(np.outer(i, i) * np.pi / N)
    assert np.max(np.abs(P[:, -1])) < 1e-14 and np.linalg.matrix_rank(P) < N
    printed = (h / 6.0) * (6.0 - 4.0 * np.sin((i - 1) * np.pi / (2 * N)))
    true = np.linalg.eigvalsh(A)
    assert np.max(np.abs(np.sort(printed) - np.sort(true))) > 1e-3
    np.testing.assert_allclose(np.sort(spectral.fourier_eigs(N, h)[0]), np.sort(true), atol=1e-15)


@pytest.mark.parametrize("stages", [1, 2])
@pytest.mark.parametrize("N", [[8], [6, 4], [4, 6, 5]])
def test_periodic_tiers_agree(stages, N):
    h = [1.0 / n for n in N]
    u0 = np.random.default_rng(sum(N)).uniform(-0.9, 0.9, tuple(reversed(N)))
    outs = [stepper.run(spectral.make_basis(t, N, h, 0.01, bc="periodic"), u0, problems.allen_cahn(), 0.1, 4,
                        stages) for t in "ABC"]
    np.testing.assert_allclose(outs[1], outs[0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(outs[2], outs[0], rtol=0, atol=1e-12)


@pytest.mark.parametrize("stages", [1, 2])
def test_single_fourier_mode_decays_like_matrix_exponential(stages):
    """f = 0: a cosine/sine product mode is an eigenvector of M^{-1} K, so both schemes
    reproduce e^{-n tau L} u0 exactly; the reference applies scipy's expm to the
    assembled matrices."""
    N, h, D, tau, n = [8, 6], [1 / 8, 1 / 6], 0.3, 0.05, 5
    X = fem.mesh(N, h, bc="periodic")
    u0 = np.cos(2 * np.pi * 2 * X[0]) * np.sin(2 * np.pi * 1 * X[1])
    M, K = fem.mass_stiffness(N, h, D, "periodic")
    L = np.linalg.solve(M.toarray(), K.toarray())
    ref = (scipy.linalg.expm(-n * tau * L) @ u0.reshape(-1)).reshape(u0.shape)
    got = stepper.run(spectral.make_basis("C", N, h, D, bc="periodic"), u0, problems.zero(), tau, n, stages)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("stages", [1, 2])
def test_constant_forcing_exact_on_the_periodic_grid(stages):
    """u-independent constant g: u(tau) = e^{-tau L} u0 + tau phi_1(-tau L) g; on a periodic grid
    the mean grows by exactly g tau per step (the constant is the zero mode)."""
    N, h, D, tau, g = [6, 5], [1 / 6, 1 / 5], 0.7, 0.2, 0.37
    u0 = np.random.default_rng(3).uniform(-1, 1, (5, 6))
    M, K = fem.mass_stiffness(N, h, D, "periodic")
    n = M.shape[0]
    # augmented exponential: d/dt [u; 1] = [[-L, g 1], [0, 0]] [u; 1]
    L = np.linalg.solve(M.toarray(), K.toarray())
    Z = np.zeros((n + 1, n + 1))
    Z[:n, :n] = -L
    Z[:n, n] = g
    ref = scipy.linalg.expm(3 * tau * Z) @ np.append(u0.reshape(-1), 1.0)
    got = stepper.run(spectral.make_basis("A", N, h, D, bc="periodic"), u0, problems.constant(g), tau, 3, stages)
    np.testing.assert_allclose(got.reshape(-1), ref[:n], rtol=0, atol=1e-13)
    np.testing.assert_allclose(got.mean() - u0.mean(), 3 * tau * g, atol=1e-13)


def test_flory_huggins_bound_root():
    g = problems.flory_huggins_bound(0.8, 1.6)
    f = problems.flory_huggins(0.8, 1.6)
    assert abs(f(0.0, None, np.array(g))) < 1e-12
    assert 0.9574 < g < 0.9576  # Example 5.3 quotes 0.9575


def test_flory_huggins_energy_of_constant_state():
    N, h = [4, 4], [0.25, 0.25]
    c = 0.3
    F = 0.4 * ((1 + c) * np.log(1 + c) + (1 - c) * np.log(1 - c)) - 0.8 * c * c
    E = norms.flory_huggins_energy(N, h, 1e-4, np.full((4, 4), c), 0.8, 1.6)
    assert abs(E - F) < 1e-15  # area 1, no gradient


def test_flory_huggins_maximum_bound_and_energy_decay():
    """Example 5.3 parameters on a small periodic 2D grid: max|u| stays within gamma and the
    discrete energy decreases at every step (both observed in Section 5.2)."""
    N, h, eps, tau = [32, 32], [1 / 32, 1 / 32], 0.01, 5 / 512
    theta, theta_c = 0.8, 1.6
    gamma = problems.flory_huggins_bound(theta, theta_c)
    u0 = np.random.default_rng(0).uniform(-0.9, 0.9, (32, 32))
    basis = spectral.make_basis("C", N, h, eps * eps, bc="periodic")
    energies, maxima = [], []

    def cb(n, t, U):
        maxima.append(float(np.max(np.abs(U))))
        energies.append(norms.flory_huggins_energy(N, h, eps * eps, U, theta, theta_c))

    stepper.run(basis, u0, problems.flory_huggins(theta, theta_c), tau, 300, 2, callback=cb)
    assert max(maxima) <= gamma
    assert np.all(np.diff(energies) <= 1e-14)
    assert maxima[-1] > 0.9  # the states have separated towards +-gamma
