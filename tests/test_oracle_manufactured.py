"""Pins for the manufactured problem u_t = D Lap u + u^2 + g (oracle.problems.mms_u2).

The forcing g is derived from the exact solution u = e^{-t} prod_a sin(pi x_a).
These pins check it against that solution by routes that never use the formula
for g:
  * finite differences of the exact solution: the residual
    u_t - D Lap u - u^2 - g vanishes at sample points in 1D, 2D and 3D, and
    plausible slips in g (the sign of the quadratic term, the dimension factor,
    the diffusion coefficient) leave a residual of order one;
  * the discrete solution converges to the exact one, at second order in h
    (the Q1 rate) and at orders one and two in tau (Theorems 3.1 and 3.2),
    measured against the exact solution rather than a same-grid fine run.
"""
import numpy as np
import pytest

from oracle import fem, norms, problems, spectral, stepper


def _second_derivative(fun, x, axis, delta):
    """Fourth-order central difference of d^2 fun / dx_axis^2 at the points x."""
    def shifted(k):
        y = [xa.copy() for xa in x]
        y[axis] = y[axis] + k * delta
        return fun(y)
    return (-shifted(2) + 16.0 * shifted(1) - 30.0 * shifted(0) + 16.0 * shifted(-1) - shifted(-2)) / (12.0 * delta ** 2)


def _residual(forcing, D, t, x, dt=1e-3, dx=1e-2):
    """u_t - D Lap u - f(t, x, u) for the exact solution, derivatives by differences."""
    u = lambda tt, y: problems.mms_u2_exact(tt, y)
    u_t = (-u(t + 2 * dt, x) + 8 * u(t + dt, x) - 8 * u(t - dt, x) + u(t - 2 * dt, x)) / (12.0 * dt)
    lap = sum(_second_derivative(lambda y: u(t, y), x, a, dx) for a in range(len(x)))
    U = u(t, x)
    return u_t - D * lap - forcing(t, x, U)


def _points(d, seed=5, n=64):
    rng = np.random.default_rng(seed)
    return [rng.uniform(0.03, 0.97, n) for _ in range(d)]


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("D", [1.0, 0.37])
@pytest.mark.parametrize("t", [0.0, 0.3, 1.7])
def test_exact_solution_satisfies_the_manufactured_equation(d, D, t):
    x = _points(d)
    r = _residual(problems.mms_u2(D), D, t, x)
    assert np.max(np.abs(r)) < 2e-6, np.max(np.abs(r))


def _slips(D, d):
    """Plausible mistakes in g, each added to the correct forcing."""
    def s_of(X):
        s = 1.0
        for xa in X:
            s = s * np.sin(np.pi * xa)
        return s

    good = problems.mms_u2(D)
    return {
        "sign of the s^2 term": lambda t, X, U: good(t, X, U) + 2.0 * np.exp(-2.0 * t) * s_of(X) ** 2,
        "dimension factor fixed at 2": lambda t, X, U: good(t, X, U) + (2 - d) * np.pi ** 2 * D * np.exp(-t) * s_of(X),
        "D halved": lambda t, X, U: good(t, X, U) - 0.5 * d * np.pi ** 2 * D * np.exp(-t) * s_of(X),
        "sign of the e^{-t} s term": lambda t, X, U: good(t, X, U) - 2.0 * (d * np.pi ** 2 * D - 1.0) * np.exp(-t) * s_of(X),
    }


@pytest.mark.parametrize("d", [1, 3])
def test_residual_check_rejects_slips_in_g(d):
    D = 0.37
    x = _points(d)
    for name, f in _slips(D, d).items():
        if name == "dimension factor fixed at 2" and d == 2:
            continue
        r = _residual(f, D, 0.3, x)
        assert np.max(np.abs(r)) > 1e-2, name


def test_converges_to_exact_solution_at_second_order_in_h():
    """EIFE2 with a small step on 2D grids 16^2 ... 64^2: the L2 error against the exact
    nodal values falls by 4 per refinement (the time error is far below)."""
    errs = []
    T, n = 0.5, 2 ** 9
    for N in (16, 32, 64):
        Ns, h = [N, N], [1.0 / N, 1.0 / N]
        b = spectral.make_basis("C", Ns, h, 1.0)
        X = fem.mesh(Ns, h)
        U = stepper.run(b, problems.mms_u2_exact(0.0, X), problems.mms_u2(1.0), T / n, n, 2)
        errs.append(norms.discrete_norms(Ns, h, U - problems.mms_u2_exact(T, X))[0])
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.05), rates
    assert errs[0] < 4e-3


@pytest.mark.parametrize("stages,order", [(1, 1.0), (2, 2.0)])
def test_temporal_orders_against_exact_solution(stages, order):
    """Theorems 3.1/3.2 on a 1D grid fine enough (16383 nodes) that the spatial error is
    below the time error: slopes of the error at T = 1 against the exact solution."""
    N, h = [16384], [1.0 / 16384]
    b = spectral.make_basis("C", N, h, 1.0)
    X = fem.mesh(N, h)
    u0 = problems.mms_u2_exact(0.0, X)
    taus, errs = [], []
    for k in range(5, 9):
        U = stepper.run(b, u0, problems.mms_u2(1.0), 2.0 ** -k, 2 ** k, stages)
        errs.append(np.max(np.abs(U - problems.mms_u2_exact(1.0, X))))
        taus.append(2.0 ** -k)
    s = np.diff(np.log(errs)) / np.diff(np.log(taus))
    assert np.all(np.abs(s - order) < 0.1), s


def test_slip_in_g_stalls_convergence():
    """With the sign of the quadratic term flipped, refining tau no longer approaches
    the exact solution (the order pins above would fail)."""
    N, h = [1024], [1.0 / 1024]
    b = spectral.make_basis("C", N, h, 1.0)
    X = fem.mesh(N, h)
    bad = _slips(1.0, 1)["sign of the s^2 term"]
    errs = []
    for k in (4, 7):
        U = stepper.run(b, problems.mms_u2_exact(0.0, X), bad, 2.0 ** -k, 2 ** k, 2)
        errs.append(np.max(np.abs(U - problems.mms_u2_exact(1.0, X))))
    assert min(errs) > 1e-2 and errs[1] > 0.5 * errs[0]
