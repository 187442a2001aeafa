"""Pins for the oracle's nonhomogeneous Dirichlet data (the extension stated at
the start of Section 4: boundary values enter the scheme as part of f) and
Example 5.2's traveling wave.

Reading: u_h = sum_interior u_i phi_i + sum_boundary g_j(t) phi_j tested with
the interior hat functions, so the load gains -Mb g'(t) - Kb g(t).  Each pin
checks the oracle against something it does not compute itself: element
quadrature over all nodes, an exact solution that the scheme must reproduce to
rounding, finite differences of the closed-form wave, and the rates of Table 4.
"""
import os

import numpy as np
import pytest

from oracle import fem, norms, problems, spectral, stepper

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table4_ex52.txt")
EPS = 0.05


@pytest.mark.parametrize("N,h,D", [([3], [0.4], 1.0), ([3, 4], [0.25, 0.4], 0.7), ([2, 3, 2], [0.5, 0.3, 0.2], 1.3)])
def test_boundary_blocks_equal_element_quadrature(N, h, D):
    Mb, Kb, Xb = fem.boundary_coupling(N, h, D)
    Mq, Kq = fem.q1_quadrature_assembly(N, h, D, all_nodes=True)
    mask = fem.boundary_nodes(N).reshape(-1)
    rows, cols = np.flatnonzero(~mask), np.flatnonzero(mask)
    np.testing.assert_allclose(Mb.toarray(), Mq[np.ix_(rows, cols)], rtol=0, atol=1e-15)
    np.testing.assert_allclose(Kb.toarray(), Kq[np.ix_(rows, cols)], rtol=0, atol=1e-13)
    assert mask.sum() == np.prod([n + 1 for n in N]) - np.prod([n - 1 for n in N])
    # the interior block of the all-node matrices is the Dirichlet pair
    M, K = fem.mass_stiffness(N, h, D)
    np.testing.assert_allclose(M.toarray(), Mq[np.ix_(rows, rows)], atol=1e-15)
    np.testing.assert_allclose(K.toarray(), Kq[np.ix_(rows, rows)], atol=1e-13)
    # boundary coordinates lie on the boundary
    for a in range(len(N)):
        assert np.all((Xb[a] >= -1e-15) & (Xb[a] <= N[a] * h[a] + 1e-15))
    on = np.zeros(len(Xb[0]), dtype=bool)
    for a in range(len(N)):
        on |= np.isclose(Xb[a], 0.0) | np.isclose(Xb[a], N[a] * h[a])
    assert on.all()


@pytest.mark.parametrize("tier", ["A", "B", "C"])
@pytest.mark.parametrize("N", [[7], [6, 5], [4, 5, 3]])
def test_linear_in_time_data_is_reproduced_exactly(tier, N):
    """f = l(x), g = t l(x), l linear: u = t l(x) is the exact solution and also the exact
    semi-discrete one (Q1 reproduces l; its stiffness annihilates it), and the load
    M^{-1}(F - Mb g' - Kb g) is linear in t, which EIFE2 integrates exactly."""
    d = len(N)
    h = [0.9 / n for n in N]
    coef = [0.3, 1.1, -0.7, 0.4][: d + 1]
    f, g, g_t, l = problems.linear_in_time_data(coef)
    b = spectral.make_basis(tier, N, h, 0.37)
    X = fem.mesh(N, h)
    tau, steps = 0.05, 6
    U = stepper.run(b, np.zeros(b.shape), f, tau, steps, 2, boundary=(g, g_t))
    ref = steps * tau * np.broadcast_to(l(X), b.shape)
    np.testing.assert_allclose(U, ref, rtol=0, atol=1e-13)


def test_linear_data_pin_sees_a_missing_term():
    """The closed form fails when either boundary term is left out (the pin is sensitive)."""
    N, h = [6, 5], [0.15, 0.18]
    f, g, g_t, l = problems.linear_in_time_data([0.3, 1.1, -0.7])
    b = spectral.make_basis("C", N, h, 0.37)
    ref = 0.3 * np.broadcast_to(l(fem.mesh(N, h)), b.shape)
    zero = lambda t, Xb: 0.0 * Xb[0]
    for bd in ((g, zero), (zero, g_t)):
        U = stepper.run(b, np.zeros(b.shape), f, 0.05, 6, 2, boundary=bd)
        assert np.max(np.abs(U - ref)) > 1e-3


def test_traveling_wave_solves_the_equation():
    u, u_t, u_x = problems.traveling_wave_solution(EPS)
    f = problems.traveling_wave(EPS)
    x = np.linspace(0.05, 1.35, 27)
    t, dt, dx = 0.013, 1e-6, 1e-4
    ut_fd = (u(t + dt, x) - u(t - dt, x)) / (2 * dt)
    ux_fd = (u(t, x + dx) - u(t, x - dx)) / (2 * dx)
    uxx_fd = (u(t, x + dx) - 2 * u(t, x) + u(t, x - dx)) / dx ** 2
    np.testing.assert_allclose(u_t(t, x), ut_fd, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(u_x(t, x), ux_fd, rtol=1e-6, atol=1e-6)
    residual = ut_fd - uxx_fd - f(t, None, u(t, x))
    assert np.max(np.abs(residual)) < 1e-3 * np.max(np.abs(ut_fd))


def _table4():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                s, nt, nx, ny, nz, l2, h1 = line.split()
                rows.append((s, int(nt), int(nx), int(ny), int(nz), float(l2), float(h1)))
    return rows


def _ex52(nx, ny, steps, stages, load="lumped"):
    u, u_t, u_x = problems.traveling_wave_solution(EPS)
    N = [nx, ny, ny]
    h = [np.sqrt(2.0) / nx, 0.125 / ny, 0.125 / ny]
    T = 3.0 * np.sqrt(2.0) * EPS / 5.0
    b = spectral.make_basis("C", N, h, 1.0)
    X = fem.mesh(N, h)
    U = stepper.run(b, u(0.0, X[0]) * np.ones(b.shape), problems.traveling_wave(EPS), T / steps, steps, stages,
                    load=load, boundary=(lambda t, Xb: u(t, Xb[0]), lambda t, Xb: u_t(t, Xb[0])))
    ex = lambda t, Y: u(t, Y[0]) + 0.0 * sum(Y[1:])
    gr = lambda t, Y: [u_x(t, Y[0]) + 0.0 * sum(Y[1:])] + [0.0 * Y[0] + 0.0 * y for y in Y[1:]]
    return norms.quadrature_errors(N, h, None, U, ex, gr, T)


def test_table4_golden_file_complete():
    rows = _table4()
    assert len(rows) == 12 and sum(r[2] <= 512 for r in rows) == 4


def test_table4_spatial_rates():
    """First two spatial rows of Table 4 (EIFE2, N_T = 1024): the oracle's continuous errors
    fall at the printed rates (L2 1.90, H1 1.11) within the intervals below; the values
    themselves depend on unstated choices (the load reading, the quadrature) and are
    compared in the design notes, not pinned."""
    rows = [r for r in _table4() if r[2] <= 128]
    errs = [_ex52(r[2], r[3], r[1], 2) for r in rows]
    l2_rate = np.log2(errs[0][0] / errs[1][0])
    h1_rate = np.log2(errs[0][1] / errs[1][1])
    printed_l2 = np.log2(rows[0][5] / rows[1][5])
    printed_h1 = np.log2(rows[0][6] / rows[1][6])
    assert 1.7 <= l2_rate <= 2.1 and 1.7 <= printed_l2 <= 2.1
    assert 0.9 <= h1_rate <= 1.3 and 0.9 <= printed_h1 <= 1.3
    # same order of magnitude as the printed errors
    for (l2, h1), r in zip(errs, rows):
        assert 0.1 < l2 / r[5] < 10 and 0.5 < h1 / r[6] < 2


def test_bench_wave_quadrature_equals_oracle_quadrature():
    """The chunked error quadrature of the Example 5.2 bench equals the oracle's on random data."""
    import bench
    u, _, u_x = problems.traveling_wave_solution(EPS)
    N = [16, 4, 3]
    h = [np.sqrt(2.0) / 16, 0.125 / 4, 0.125 / 3]
    U = np.random.default_rng(0).uniform(0.0, 1.0, (2, 3, 15))
    ex = lambda t, Y: u(t, Y[0]) + 0.0 * sum(Y[1:])
    gr = lambda t, Y: [u_x(t, Y[0]) + 0.0 * sum(Y[1:])] + [0.0 * Y[0] + 0.0 * y for y in Y[1:]]
    got = bench.q1_errors_wave(U, N, h, 0.02, EPS, zchunk=2)
    ref = norms.quadrature_errors(N, h, None, U, ex, gr, 0.02)
    np.testing.assert_allclose(got, ref, rtol=1e-13)
