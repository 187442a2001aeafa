"""Pins for variable step sizes tau_n (Section 2.2 defines the schemes with
t_{n+1} = t_n + tau_n and every operator function formed with tau_n).

Each pin uses something the stepper does not compute itself: the matrix
exponential of the assembled operator (augmented for forcing), for which
EIFE1 is exact with constant forcing and EIFE2 with forcing affine in t, at
any step sequence; and the observed order on graded step sequences.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import fem, norms, problems, spectral, stepper


def _augmented(N, h, D, c0, c1, T, u0):
    """Exact solution of M u' + K u = (c0 + c1 t) prod(h) 1 (the lumped load of a
    u- and x-independent forcing) at time T, via expm of an augmented system."""
    M, K = fem.mass_stiffness(N, h, D)
    n = M.shape[0]
    L = np.linalg.solve(M.toarray(), K.toarray())
    v = np.linalg.solve(M.toarray(), np.full(n, float(np.prod(h))))
    # state [u; 1; t]: u' = -L u + (c0 + c1 t) v, 1' = 0, t' = 1
    Z = np.zeros((n + 2, n + 2))
    Z[:n, :n] = -L
    Z[:n, n] = c0 * v
    Z[:n, n + 1] = c1 * v
    Z[n + 1, n] = 1.0
    y = scipy.linalg.expm(T * Z) @ np.concatenate([u0.reshape(-1), [1.0, 0.0]])
    return y[:n].reshape(u0.shape)


TAUS = np.random.default_rng(4).uniform(0.02, 0.3, 9)


@pytest.mark.parametrize("tier", ["A", "B", "C"])
def test_eife2_exact_for_affine_forcing_at_random_steps(tier):
    N, h, D = [6, 5], [1 / 6, 1 / 5], 0.6
    u0 = np.random.default_rng(1).uniform(-1, 1, (4, 5))
    b = spectral.make_basis(tier, N, h, D)
    got = stepper.run(b, u0, problems.affine_t(0.4, -1.3), TAUS, len(TAUS), 2, c2=0.37)
    ref = _augmented(N, h, D, 0.4, -1.3, TAUS.sum(), u0)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_eife1_exact_for_constant_forcing_at_random_steps():
    N, h, D = [7, 4, 3], [1 / 7, 1 / 4, 1 / 3], 0.45
    u0 = np.random.default_rng(2).uniform(-1, 1, (2, 3, 6))
    b = spectral.make_basis("C", N, h, D)
    got = stepper.run(b, u0, problems.constant(0.8), TAUS, len(TAUS), 1)
    ref = _augmented(N, h, D, 0.8, 0.0, TAUS.sum(), u0)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_times_follow_the_running_sum():
    """With forcing affine in t, EIFE1 is not exact, and its error depends on the t_n it
    used: using t0 + n * mean(tau) instead of the running sum changes the result."""
    N, h, D = [8], [1 / 8], 0.3
    u0 = np.zeros((7,))
    b = spectral.make_basis("C", N, h, D)
    f = problems.affine_t(0.0, 1.0)
    seen = []
    stepper.run(b, u0, f, TAUS, len(TAUS), 1, t0=0.25, callback=lambda n, t, U: seen.append(t))
    np.testing.assert_allclose(seen, 0.25 + np.cumsum(TAUS), rtol=0, atol=1e-15)


@pytest.mark.parametrize("stages,order", [(1, 1.0), (2, 2.0)])
def test_order_on_graded_steps(stages, order):
    """Geometrically graded steps (ratio 1.05) refined by halving every step: the error
    against a fine uniform reference falls at the scheme's order."""
    N, h, D = [16, 16], [1 / 16, 1 / 16], 0.01
    u0 = np.random.default_rng(3).uniform(-0.9, 0.9, (15, 15))
    b = spectral.make_basis("C", N, h, D)
    f = problems.allen_cahn()
    base = 1.05 ** np.arange(32)
    base = base / base.sum()  # T = 1
    ref = stepper.run(b, u0, f, 1.0 / 8192, 8192, 2)
    errs = []
    for k in range(3):
        taus = np.repeat(base / 2 ** k, 2 ** k)
        U = stepper.run(b, u0, f, taus, len(taus), stages)
        errs.append(norms.discrete_norms(N, h, U - ref)[0])
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.25), rates


def test_uniform_sequence_equals_scalar_step():
    N, h = [9, 7], [1 / 9, 1 / 7]
    u0 = np.random.default_rng(5).uniform(-0.9, 0.9, (6, 8))
    b = spectral.make_basis("C", N, h, 0.02)
    a = stepper.run(b, u0, problems.allen_cahn(), 0.05, 6, 2)
    c = stepper.run(b, u0, problems.allen_cahn(), [0.05] * 6, 6, 2)
    np.testing.assert_allclose(a, c, rtol=0, atol=1e-15)
