"""GPU parity for variable step sizes tau_n (Section 2.2) against the FP64
oracle, whose variable-step stepper is pinned by the CPU tests (exactness
against the matrix exponential at random step sequences, graded-step orders).
Tolerances as everywhere: relative max-norm 1e-12 (FP64), 1e-5 (FP32).
"""
import numpy as np
import pytest

import seeded_inputs
from oracle import fem, problems, spectral, stepper

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _eife():
    import paper_2209_11922_amd as eife
    return eife


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _taus(seed, n, lo, hi):
    return np.random.default_rng(seed).uniform(lo, hi, n)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("stages", [2, 1])
@pytest.mark.parametrize("N", [[64, 48], [16, 12, 18], [256, 256, 8]], ids=["2d", "3d-mixed", "3d-fast"])
def test_allen_cahn_random_steps_match_oracle(N, stages, dtype):
    eife = _eife()
    h = [1.0 / n for n in N]
    u0 = seeded_inputs.uniform_field(3, N)
    taus = _taus(7, 9, 0.005, 0.05)
    g = eife.Grid(N, h, 1e-3, dtype)
    g.set_phi(0.01, stages)
    u = torch.tensor(u0, dtype=g.torch_dtype, device="cuda")
    g.step_variable(u, taus, eife.F_ALLEN_CAHN, 0.0)
    torch.cuda.synchronize()
    got = u.double().cpu().numpy()
    g.close()
    ref = stepper.run(spectral.make_basis("C", N, h, 1e-3), u0, problems.allen_cahn(), taus, len(taus), stages)
    err = _rel(got, ref)
    print(f"variable steps {N} EIFE{stages} {dtype}: {err:.2e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("stages", [2, 1])
def test_time_dependent_forcing_uses_the_running_sum(stages):
    """The manufactured forcing depends on t: t_n and t_n + c2 tau_n must follow the steps."""
    eife = _eife()
    N = [32, 24]
    h = [1.0 / n for n in N]
    X = fem.mesh(N, h)
    u0 = problems.mms_u2_exact(0.3, X)
    taus = _taus(11, 12, 0.002, 0.04)
    g = eife.Grid(N, h, 0.5, "f64")
    g.set_c2(0.3)
    g.set_phi(0.01, stages)
    u = torch.tensor(u0, device="cuda")
    g.step_variable(u, taus, eife.F_MMS_U2, 0.3)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    g.close()
    ref = stepper.run(spectral.make_basis("C", N, h, 0.5), u0, problems.mms_u2(0.5), taus, len(taus), stages,
                      c2=0.3, t0=0.3)
    assert _rel(got, ref) <= 1e-12


def test_equal_steps_give_the_bits_of_eife_step():
    eife = _eife()
    N = [128, 96]
    h = [1.0 / n for n in N]
    u0 = seeded_inputs.uniform_field(5, N)
    outs = []
    for variable in (False, True):
        g = eife.Grid(N, h, 2e-3, "f32")
        g.set_phi(0.02, 2)
        u = torch.tensor(u0, dtype=torch.float32, device="cuda")
        if variable:
            g.step_variable(u, [0.02] * 7, eife.F_ALLEN_CAHN, 0.1)
        else:
            g.step(u, 7, eife.F_ALLEN_CAHN, 0.1)
        torch.cuda.synchronize()
        outs.append(u.cpu())
        g.close()
    assert torch.equal(outs[0], outs[1])


def test_more_steps_than_one_chunk():
    """1100 steps cross two chunk boundaries of the per-step tables (512 steps each)."""
    eife = _eife()
    N = [24, 18]
    h = [1.0 / n for n in N]
    u0 = seeded_inputs.uniform_field(9, N)
    taus = 0.001 * (1.0 + 0.5 * np.sin(np.arange(1100)))
    g = eife.Grid(N, h, 1e-3, "f64")
    g.set_phi(0.01, 2)
    u = torch.tensor(u0, device="cuda")
    g.step_variable(u, taus, eife.F_ALLEN_CAHN)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    g.close()
    ref = stepper.run(spectral.make_basis("C", N, h, 1e-3), u0, problems.allen_cahn(), taus, len(taus), 2)
    assert _rel(got, ref) <= 1e-12


def test_periodic_and_split_bf16_variable_steps():
    eife = _eife()
    taus = _taus(13, 6, 0.01, 0.05)
    for N in ([32, 36], [256, 128]):  # generic and wave-local periodic passes
        h = [1.0 / n for n in N]
        u0 = np.random.default_rng(2).uniform(-0.9, 0.9, tuple(reversed(N)))
        g = eife.Grid(N, h, 1e-3, "f64", bc=eife.BC_PERIODIC)
        g.set_phi(0.01, 2)
        u = torch.tensor(u0, device="cuda")
        g.step_variable(u, taus, eife.F_ALLEN_CAHN)
        torch.cuda.synchronize()
        ref = stepper.run(spectral.make_basis("C", N, h, 1e-3, bc="periodic"), u0, problems.allen_cahn(), taus,
                          len(taus), 2)
        assert _rel(u.cpu().numpy(), ref) <= 1e-12
        g.close()
    # matrix-core transform: its own error bound (split-BF16 products)
    N = [64, 64]
    h = [1.0 / 64] * 2
    u0 = seeded_inputs.uniform_field(4, N)
    g = eife.Grid(N, h, 1e-3, "f32")
    g.set_transform(eife.binding.TX_GEMM_SPLITBF16)
    g.set_phi(0.01, 2)
    u = torch.tensor(u0, dtype=torch.float32, device="cuda")
    g.step_variable(u, taus, eife.F_ALLEN_CAHN)
    torch.cuda.synchronize()
    ref = stepper.run(spectral.make_basis("C", N, h, 1e-3), u0, problems.allen_cahn(), taus, len(taus), 2)
    assert _rel(u.double().cpu().numpy(), ref) <= 2e-4
    g.close()


def test_variable_step_argument_errors():
    eife = _eife()
    g = eife.Grid([16, 16], [1 / 16, 1 / 16], 1e-3, "f64")
    u = torch.zeros(15 * 15, dtype=torch.float64, device="cuda")
    with pytest.raises(eife.EIFEError) as e:  # no eife_set_phi yet
        g.step_variable(u, [0.01], eife.F_ALLEN_CAHN)
    assert e.value.code == -4
    g.set_phi(0.01, 2)
    for bad in ([0.01, 0.0], [0.01, -1.0], [float("nan")]):
        with pytest.raises(eife.EIFEError) as e:
            g.step_variable(u, bad, eife.F_ALLEN_CAHN)
        assert e.value.code == -1
    with pytest.raises(eife.EIFEError) as e:
        g.step_variable(u, [0.01], 42)
    assert e.value.code == -1
    g.step_variable(u, [], eife.F_ALLEN_CAHN)
    g.close()
