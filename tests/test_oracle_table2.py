"""Pin the oracle to the errors printed in Table 2 (Example 5.1).

Readings (each listed in the design notes):
* the load is lumped, F_i = f(u_i) * prod(h) (Section 4's load tensor);
* errors are the discrete M- and (M + K_1)-norms of the nodal error for the
  temporal rows, and the 4x4-Gauss continuous L2 error for the spatial rows;
* the EIFE1 temporal rows are reproduced with 2 N_T uniform steps on [0, 1],
  not N_T: with N_T steps every EIFE1 error is about twice the printed one,
  while the EIFE2 rows match with N_T as printed.
"""
import os

import numpy as np
import pytest

from oracle import fem, norms, problems, spectral, stepper

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_ex51.txt")


def _rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            s, nt, nx, ny, l2, h1 = line.split()
            rows.append((s, int(nt), int(nx), int(ny), float(l2), float(h1)))
    return rows


ROWS = _rows()
SPATIAL = [r for r in ROWS if r[2] <= 64]
TEMPORAL = [r for r in ROWS if r[2] == 2048]


def _solve(nx, ny, steps, stages):
    N = [nx, ny]
    h = [2.0 / nx, 1.0 / ny]
    b = spectral.make_basis("C", N, h, problems.EX51_D)
    X = fem.mesh(N, h, problems.EX51_ORIGIN)
    u0 = problems.ex51_exact(0.0, X)
    U = stepper.run(b, u0, problems.ex51(), 1.0 / steps, steps, stages, 0.5,
                    origin=problems.EX51_ORIGIN)
    return N, h, X, U


def test_golden_file_complete():
    assert len(SPATIAL) == 4 and len(TEMPORAL) == 8


@pytest.mark.slow
@pytest.mark.parametrize("row", TEMPORAL, ids=lambda r: f"{r[0]}-NT{r[1]}")
def test_temporal_rows(row):
    scheme, nt, nx, ny, l2, h1 = row
    stages = 1 if scheme == "EIFE1" else 2
    steps = 2 * nt if stages == 1 else nt
    N, h, X, U = _solve(nx, ny, steps, stages)
    e = problems.ex51_exact(1.0, X) - U
    el2, eh1, _ = norms.discrete_norms(N, h, e)
    assert el2 == pytest.approx(l2, rel=0.01)
    assert eh1 == pytest.approx(h1, rel=0.005)


def test_eife1_with_printed_step_count_misses_the_printed_row():
    """Supports the 2 N_T reading: at N_T steps EIFE1 misses the printed row by 60 percent."""
    scheme, nt, nx, ny, l2, h1 = [r for r in TEMPORAL if r[0] == "EIFE1"][0]
    N, h, X, U = _solve(nx, ny, nt, 1)
    el2, _, _ = norms.discrete_norms(N, h, problems.ex51_exact(1.0, X) - U)
    assert 1.5 < el2 / l2 < 2.2


@pytest.mark.parametrize("row", SPATIAL, ids=lambda r: f"{r[2]}x{r[3]}")
def test_spatial_rows_l2(row):
    scheme, nt, nx, ny, l2, h1 = row
    N, h, X, U = _solve(nx, ny, nt, 2)
    ql2, qh1 = norms.quadrature_errors_2d(N, h, problems.EX51_ORIGIN, U, problems.ex51_exact,
                                         problems.ex51_exact_grad, 1.0)
    # the paper names no quadrature; the continuous L2 error lands within 4%
    assert ql2 == pytest.approx(l2, rel=0.04)


def test_spatial_l2_rates_near_two():
    errs = []
    for scheme, nt, nx, ny, l2, h1 in SPATIAL:
        N, h, X, U = _solve(nx, ny, nt, 2)
        errs.append(norms.quadrature_errors_2d(N, h, problems.EX51_ORIGIN, U, problems.ex51_exact,
                                               problems.ex51_exact_grad, 1.0)[0])
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    printed = np.log2(np.array([r[4] for r in SPATIAL[:-1]]) / np.array([r[4] for r in SPATIAL[1:]]))
    np.testing.assert_allclose(rates, printed, atol=0.12)
