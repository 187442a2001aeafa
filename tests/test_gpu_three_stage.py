"""GPU parity for the three-stage scheme of eq. (2.2) (nodes 0, c2, c3) against
the FP64 oracle's general s-stage step (oracle/erk.py), which the CPU tests pin
to the consistency conditions of eq. (2.3), the EIFE1/EIFE2 formulas, the
matrix exponential (exactness for quadratic-in-t forcing) and observed orders.
Tolerances as everywhere: relative max-norm 1e-12 (FP64), 1e-5 (FP32).
"""
import numpy as np
import pytest

import seeded_inputs
from oracle import erk, fem, problems, spectral

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _eife():
    import paper_2209_11922_amd as eife
    return eife


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _run(N, D, u0, tau, steps, nodes, fkind, dtype, bc=0, t0=0.0, variable=None):
    eife = _eife()
    g = eife.Grid(N, [1.0 / n for n in N], D, dtype, bc=bc)
    g.set_nodes3(nodes[1], nodes[2])
    g.set_phi(tau, 3)
    u = torch.tensor(np.ascontiguousarray(u0), dtype=g.torch_dtype, device="cuda")
    if variable is None:
        g.step(u, steps, fkind, t0)
    else:
        g.step_variable(u, variable, fkind, t0)
    torch.cuda.synchronize()
    out = u.double().cpu().numpy()
    g.close()
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nodes", [(0.0, 1 / 3, 2 / 3), (0.0, 0.5, 1.0)], ids=["thirds", "simpson"])
@pytest.mark.parametrize("N", [[64], [64, 48], [16, 12, 18], [128, 64, 32]],
                         ids=["1d", "2d", "3d-mixed", "3d-fast-rows"])
def test_allen_cahn_matches_oracle(N, nodes, dtype):
    eife = _eife()
    h = [1.0 / n for n in N]
    u0 = seeded_inputs.uniform_field(21, N)
    got = _run(N, 1e-3, u0, 0.02, 6, nodes, eife.F_ALLEN_CAHN, dtype)
    ref = erk.run(spectral.make_basis("C", N, h, 1e-3), u0, problems.allen_cahn(), 0.02, 6, list(nodes))
    err = _rel(got, ref)
    print(f"three stages {N} {nodes} {dtype}: {err:.2e}")
    assert err <= TOL[dtype]


def test_time_dependent_forcing_and_variable_steps():
    """Manufactured forcing (depends on t) from t0 > 0: the stage times t_n + c_i tau_n, uniform
    and varying steps."""
    eife = _eife()
    N = [32, 24]
    h = [1.0 / n for n in N]
    u0 = problems.mms_u2_exact(0.2, fem.mesh(N, h))
    b = spectral.make_basis("C", N, h, 0.5)
    nodes = (0.0, 0.3, 0.8)
    got = _run(N, 0.5, u0, 0.03, 5, nodes, eife.F_MMS_U2, "f64", t0=0.2)
    ref = erk.run(b, u0, problems.mms_u2(0.5), 0.03, 5, list(nodes), t0=0.2)
    assert _rel(got, ref) <= 1e-12
    taus = np.random.default_rng(3).uniform(0.005, 0.05, 8)
    got = _run(N, 0.5, u0, 0.03, 0, nodes, eife.F_MMS_U2, "f64", t0=0.2, variable=taus)
    ref = erk.run(b, u0, problems.mms_u2(0.5), taus, 8, list(nodes), t0=0.2)
    assert _rel(got, ref) <= 1e-12


@pytest.mark.parametrize("N", [[32, 36], [128, 256]], ids=["generic", "wave-local-rows"])
def test_periodic_three_stages(N):
    eife = _eife()
    h = [1.0 / n for n in N]
    u0 = np.random.default_rng(4).uniform(-0.9, 0.9, tuple(reversed(N)))
    got = _run(N, 1e-3, u0, 0.02, 6, (0.0, 1 / 3, 2 / 3), eife.F_ALLEN_CAHN, "f64", bc=eife.BC_PERIODIC)
    ref = erk.run(spectral.make_basis("C", N, h, 1e-3, bc="periodic"), u0, problems.allen_cahn(), 0.02, 6,
                  [0.0, 1 / 3, 2 / 3])
    assert _rel(got, ref) <= 1e-12


def test_affine_forcing_matches_oracle():
    """u-independent forcing c0 + c1 t, which the scheme integrates exactly (the CPU pins tie
    the oracle to the matrix exponential for forcing up to degree 2)."""
    eife = _eife()
    N = [16, 12]
    h = [1 / 16, 1 / 12]
    u0 = np.random.default_rng(9).uniform(-1, 1, (11, 15))
    g = eife.Grid(N, h, 0.3, "f64")
    g.set_forcing(0.5, 2.0)
    g.set_phi(0.1, 3)
    u = torch.tensor(u0, device="cuda")
    g.step(u, 5, eife.F_AFFINE_T, 0.0)
    torch.cuda.synchronize()
    ref = erk.run(spectral.make_basis("C", N, h, 0.3), u0, problems.affine_t(0.5, 2.0), 0.1, 5,
                  [0.0, 1 / 3, 2 / 3])
    assert _rel(u.cpu().numpy(), ref) <= 1e-12
    g.close()


def test_three_stage_argument_errors():
    eife = _eife()
    g = eife.Grid([32, 32], [1 / 32, 1 / 32], 1e-3, "f32")
    for c2, c3 in ((0.0, 0.5), (0.6, 0.5), (0.5, 0.5), (0.3, 1.2)):
        with pytest.raises(eife.EIFEError) as e:
            g.set_nodes3(c2, c3)
        assert e.value.code == -1
    with pytest.raises(eife.EIFEError) as e:
        g.set_phi(0.01, 4)
    assert e.value.code == -1
    g.set_phi(0.01, 3)
    u = torch.zeros(31 * 31, dtype=torch.float32, device="cuda")
    g.step(u, 1, eife.F_ALLEN_CAHN)
    g.set_nodes3(0.4, 0.9)
    with pytest.raises(eife.EIFEError) as e:  # nodes changed: set_phi again
        g.step(u, 1, eife.F_ALLEN_CAHN)
    assert e.value.code == -4
    g.set_phi(0.01, 3)
    g.set_transform(eife.binding.TX_GEMM_SPLITBF16)
    with pytest.raises(eife.EIFEError) as e:
        g.step(u, 1, eife.F_ALLEN_CAHN)
    assert e.value.code == -3
    g.close()
