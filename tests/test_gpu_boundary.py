"""GPU parity for nonhomogeneous Dirichlet data (start of Section 4: the boundary
values enter as part of f) on Example 5.2's traveling wave, against the FP64
oracle, whose boundary term is pinned by the CPU tests (all-node element
quadrature, an exactly reproduced linear-in-time solution).  Tolerances as
everywhere: relative max-norm 1e-12 (FP64), 1e-5 (FP32).
"""
import numpy as np
import pytest

from oracle import fem, problems, spectral, stepper

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
EPS = 0.05
T_END = 3.0 * np.sqrt(2.0) * EPS / 5.0


def _eife():
    import paper_2209_11922_amd as eife
    return eife


def _geometry(N):
    lengths = [np.sqrt(2.0), 0.125, 0.125][: len(N)]
    return [L / n for L, n in zip(lengths, N)]


def _u0(N, h):
    u, _, _ = problems.traveling_wave_solution(EPS)
    X = fem.mesh(N, h)
    return u(0.0, X[0]) * np.ones(tuple(n - 1 for n in reversed(N)))


def _gpu(N, h, u0, tau, steps, stages, dtype):
    eife = _eife()
    g = eife.Grid(N, h, 1.0, dtype)
    g.set_forcing(EPS, 0.0)
    g.set_phi(tau, stages)
    u = torch.tensor(np.ascontiguousarray(u0), dtype=g.torch_dtype, device="cuda")
    g.step(u, steps, eife.F_TRAVELING_WAVE, 0.0)
    torch.cuda.synchronize()
    out = u.double().cpu().numpy()
    g.close()
    return out


def _oracle(N, h, u0, tau, steps, stages):
    u, u_t, _ = problems.traveling_wave_solution(EPS)
    b = spectral.make_basis("C", N, h, 1.0)
    return stepper.run(b, u0, problems.traveling_wave(EPS), tau, steps, stages,
                       boundary=(lambda t, Xb: u(t, Xb[0]), lambda t, Xb: u_t(t, Xb[0])))


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("stages", [2, 1])
@pytest.mark.parametrize("N", [[256], [64, 8], [64, 4, 4], [96, 6, 6], [128, 8, 8], [36, 12, 8]],
                         ids=["1d", "2d", "3d-64x4x4", "3d-mixed-radix", "3d-128x8x8", "3d-ragged"])
def test_traveling_wave_matches_oracle(N, stages, dtype):
    h = _geometry(N)
    u0 = _u0(N, h)
    tau, steps = T_END / 64, 16
    got = _gpu(N, h, u0, tau, steps, stages, dtype)
    ref = _oracle(N, h, u0, tau, steps, stages)
    err = _rel(got, ref)
    print(f"traveling wave {N} EIFE{stages} {dtype}: {err:.2e}")
    assert err <= TOL[dtype]


def test_table4_first_spatial_row_matches_oracle():
    """The configuration of Table 4's first spatial row (64 x 4 x 4, N_T = 1024, EIFE2), run to T."""
    N = [64, 4, 4]
    h = _geometry(N)
    u0 = _u0(N, h)
    got = _gpu(N, h, u0, T_END / 1024, 1024, 2, "f64")
    ref = _oracle(N, h, u0, T_END / 1024, 1024, 2)
    assert _rel(got, ref) <= 1e-12


def test_front_stays_inside_the_shell_bounds():
    """The discrete wave stays within [0, 1] up to the scheme error and moves right at speed s."""
    N = [256]
    h = _geometry(N)
    u0 = _u0(N, h)
    got = _gpu(N, h, u0, T_END / 256, 256, 2, "f64")
    u, _, _ = problems.traveling_wave_solution(EPS)
    x = fem.mesh(N, h)[0]
    assert np.max(np.abs(got - u(T_END, x))) < 1e-2
    assert -1e-3 < got.min() and got.max() < 1 + 1e-3


def test_traveling_wave_argument_errors():
    eife = _eife()
    g = eife.Grid([32, 8], [0.05, 0.02], 1.0, "f64", bc=eife.BC_PERIODIC)
    g.set_forcing(EPS, 0.0)
    g.set_phi(0.001, 2)
    u = torch.zeros(32 * 8, dtype=torch.float64, device="cuda")
    with pytest.raises(eife.EIFEError) as e:
        g.step(u, 1, eife.F_TRAVELING_WAVE)
    assert e.value.code == -3
    g.close()
    g = eife.Grid([32, 8], [0.05, 0.02], 1.0, "f64")
    g.set_phi(0.001, 2)
    u = torch.zeros(31 * 7, dtype=torch.float64, device="cuda")
    with pytest.raises(eife.EIFEError) as e:  # eps = c0 not set
        g.step(u, 1, eife.F_TRAVELING_WAVE)
    assert e.value.code == -1
    g.set_forcing(EPS, 0.0)
    g.set_load(eife.LOAD_NODAL)
    with pytest.raises(eife.EIFEError) as e:
        g.step(u, 1, eife.F_TRAVELING_WAVE)
    assert e.value.code == -3
    g.set_load(eife.LOAD_LUMPED)
    g.step(u, 1, eife.F_TRAVELING_WAVE)
    g.close()


def _table4_rows():
    import os
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "table4_ex52.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                s, nt, nx, ny, nz, l2, h1 = line.split()
                rows.append((s, int(nt), int(nx), int(ny), int(nz), float(l2), float(h1)))
    return rows


@pytest.mark.parametrize("row", [r for r in _table4_rows() if r[2] == 1024 and r[1] <= 32][:3],
                         ids=lambda r: f"{r[0]}-NT{r[1]}")
def test_table4_temporal_rows(row):
    """Table 4's temporal rows (1024 x 64 x 64, where the time error dominates): the continuous
    L2 error of the GPU solution lands within 5 percent of the printed value (all eight rows do,
    per the Example 5.2 bench; three are run here)."""
    import bench
    scheme, nt, nx, ny, nz, l2_printed, _ = row
    N = [nx, ny, nz]
    h = _geometry(N)
    got = _gpu(N, h, _u0(N, h), T_END / nt, nt, 1 if scheme == "EIFE1" else 2, "f64")
    l2, _ = bench.q1_errors_wave(got, N, h, T_END, EPS)
    print(f"{scheme} N_T={nt}: L2 {l2:.4e} (printed {l2_printed:.4e})")
    assert l2 == pytest.approx(l2_printed, rel=0.05)
