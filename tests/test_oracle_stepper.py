"""Pins for the oracle's EIFE1/EIFE2 steppers (Section 2.2, eqs. (2.13)-(2.14)).

Each pin checks the stepper against something other than its own formulas:
the matrix exponential of an augmented system (scipy.linalg.expm), other
eigen-bases, observed convergence orders (Theorems 3.1 and 3.2) and the
maximum bound principle of the Allen-Cahn equation.
"""
import numpy as np
import pytest
import scipy.linalg

import seeded_inputs
from oracle import fem, problems, spectral, stepper


def _L_dense(N, h, D):
    M, K = fem.mass_stiffness(N, h, D)
    M = M.toarray()
    return M, np.linalg.solve(M, K.toarray())


@pytest.mark.parametrize("stages", [1, 2])
@pytest.mark.parametrize("load", ["lumped", "nodal"])
@pytest.mark.parametrize("N,h", [([7, 5], [1.0 / 7, 0.21]), ([5, 4, 6], [0.2, 0.25, 1.0 / 6])])
def test_tiers_agree(stages, load, N, h):
    D = 0.3
    u0 = seeded_inputs.uniform_field(3, N)
    outs = []
    for tier in "ABC":
        b = spectral.make_basis(tier, N, h, D)
        outs.append(stepper.run(b, u0, problems.allen_cahn(), 0.05, 6, stages, 0.5,
                                load=load))
    scale = np.max(np.abs(outs[0]))
    for o in outs[1:]:
        assert np.max(np.abs(o - outs[0])) / scale < 1e-12


@pytest.mark.parametrize("N,h,D", [([9, 6], [1.0 / 9, 1.0 / 6], 0.8), ([5, 6, 4], [0.2, 1 / 6, 0.25], 0.1)])
@pytest.mark.parametrize("stages", [1, 2])
def test_single_sine_mode_decays_like_matrix_exponential(N, h, D, stages):
    """f = 0: u^n = exp(-n tau M^{-1} K) u0 for any tau; a nodal sine is an eigenvector."""
    X = fem.mesh(N, h)
    modes = [1, 2, 3][: len(N)]
    u0 = np.ones(tuple(n - 1 for n in reversed(N)))
    for a, x in enumerate(X):
        u0 = u0 * np.sin(modes[a] * np.pi * x / (N[a] * h[a]))
    M, L = _L_dense(N, h, D)
    for tau, n in [(0.01, 5), (0.7, 3)]:
        ref = scipy.linalg.expm(-n * tau * L) @ u0.reshape(-1)
        # the decay factor is that of a single eigenvalue
        flat = u0.reshape(-1)
        big = np.abs(flat) > 0.1 * np.max(np.abs(flat))
        ratio = ref[big] / flat[big]
        assert np.ptp(ratio) < 1e-12 * max(1.0, abs(ratio[0]))
        for tier in "AC":
            b = spectral.make_basis(tier, N, h, D)
            got = stepper.run(b, u0, problems.zero(), tau, n, stages)
            np.testing.assert_allclose(got.reshape(-1), ref, rtol=1e-12, atol=1e-14 * np.max(np.abs(u0)))


def _augmented_exact(N, h, D, u0, g0, g1, t0, tau, load):
    """Exact solution at t0 + tau of u' = -L u + P_h(g0 + t g1) via expm of [[-L, b1, b0], [0,0,1], [0,0,0]]."""
    M, L = _L_dense(N, h, D)
    n = L.shape[0]
    ones = np.ones(n)
    if load == "lumped":
        b = np.linalg.solve(M, ones * float(np.prod(h)))
    else:
        b = ones
    Z = np.zeros((n + 2, n + 2))
    Z[:n, :n] = -L
    Z[:n, n] = g1 * b
    Z[:n, n + 1] = g0 * b
    Z[n, n + 1] = 1.0
    y0 = np.concatenate([u0.reshape(-1), [t0, 1.0]])
    return (scipy.linalg.expm(tau * Z) @ y0)[:n]


@pytest.mark.parametrize("load", ["lumped", "nodal"])
@pytest.mark.parametrize("N,h", [([6, 5], [1 / 6, 0.2]), ([4, 3, 5], [0.25, 1 / 3, 0.2])])
def test_constant_forcing_is_exact_for_both_schemes(load, N, h):
    """Order conditions (eq. (2.11)): forcing independent of u and t is integrated exactly."""
    D = 0.6
    u0 = seeded_inputs.uniform_field(11, N)
    tau = 0.3
    ref = _augmented_exact(N, h, D, u0, 1.7, 0.0, 0.0, tau, load)
    for stages in (1, 2):
        for tier in "AC":
            b = spectral.make_basis(tier, N, h, D)
            got = stepper.run(b, u0, problems.constant(1.7), tau, 1, stages, 0.5, load=load)
            np.testing.assert_allclose(got.reshape(-1), ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("c2", [0.5, 1.0, 0.3])
@pytest.mark.parametrize("N,h", [([6, 5], [1 / 6, 0.2]), ([4, 3, 5], [0.25, 1 / 3, 0.2])])
def test_affine_in_time_forcing_exact_for_eife2_only(c2, N, h):
    D = 0.6
    u0 = seeded_inputs.uniform_field(12, N)
    tau, t0 = 0.25, 0.4
    g0, g1 = 0.9, -2.3
    ref = _augmented_exact(N, h, D, u0, g0, g1, t0, tau, "lumped")
    b = spectral.make_basis("A", N, h, D)
    got2 = stepper.run(b, u0, problems.affine_t(g0, g1), tau, 1, 2, c2, t0=t0)
    np.testing.assert_allclose(got2.reshape(-1), ref, rtol=0, atol=1e-13)
    got1 = stepper.run(b, u0, problems.affine_t(g0, g1), tau, 1, 1, t0=t0)
    assert np.max(np.abs(got1.reshape(-1) - ref)) > 1e-4


def _slopes(taus, errs):
    lt, le = np.log(taus), np.log(errs)
    return np.diff(le) / np.diff(lt)


@pytest.mark.parametrize("stages,order", [(1, 1.0), (2, 2.0)])
def test_temporal_order_manufactured_problem(stages, order):
    """Theorems 3.1/3.2: first and second order in time (same-grid fine reference)."""
    N = [32, 32]
    h = [1 / 32, 1 / 32]
    D = 1.0
    b = spectral.make_basis("C", N, h, D)
    X = fem.mesh(N, h)
    u0 = problems.mms_u2_exact(0.0, X)
    f = problems.mms_u2(D)
    ref = stepper.run(b, u0, f, 2.0 ** -13, 2 ** 13, 2)
    taus, errs = [], []
    for k in range(4, 11):
        tau = 2.0 ** -k
        U = stepper.run(b, u0, f, tau, 2 ** k, stages)
        errs.append(np.max(np.abs(U - ref)))
        taus.append(tau)
    s = _slopes(np.array(taus), np.array(errs))
    assert np.all(np.abs(s[-3:] - order) < 0.1), s


def test_allen_cahn_maximum_bound_long_run():
    """The Allen-Cahn solution stays in [-1, 1] over a long run (maximum bound principle)."""
    N = [64, 64]
    h = [1 / 64, 1 / 64]
    eps = 0.05
    b = spectral.make_basis("C", N, h, eps * eps)
    u0 = seeded_inputs.uniform_field(0, N)
    peak = [0.0]

    def cb(n, t, U):
        peak[0] = max(peak[0], float(np.max(np.abs(U))))

    stepper.run(b, u0, problems.allen_cahn(), 0.01, 3000, 2, callback=cb)
    assert 0.99 < peak[0] <= 1.0


def test_large_step_stays_bounded():
    """No step-size restriction (remark after Theorem 3.2): tau = 0.1 stays bounded."""
    N = [64, 64]
    h = [1 / 64, 1 / 64]
    b = spectral.make_basis("C", N, h, 0.05 ** 2)
    u0 = seeded_inputs.uniform_field(1, N)
    U = stepper.run(b, u0, problems.allen_cahn(), 0.1, 300, 2)
    assert np.all(np.isfinite(U)) and np.max(np.abs(U)) <= 1.0 + 1e-12


def test_stepper_rejects_bad_arguments():
    b = spectral.make_basis("C", [4, 4], [0.25, 0.25], 1.0)
    u0 = np.zeros((3, 3))
    with pytest.raises(ValueError):
        stepper.run(b, u0, problems.zero(), 0.1, 1, 3)
    with pytest.raises(ValueError):
        stepper.run(b, u0, problems.zero(), 0.1, 1, 2, c2=0.0)
