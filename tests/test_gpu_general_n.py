"""GPU parity for grids whose FFT length has prime factors above 7.

Section 4's sine (and, at its end, Fourier) diagonalisation holds for any
number of intervals N; the generic passes factor the FFT length into radices
8/4/2/3/5/7 and run each remaining prime factor as a direct-DFT Stockham
stage.  Compared with the FP64 oracle (library type-I sine / real Fourier
transforms with closed-form eigenvalues) at the tolerances of the other
parity tests: FP64 1e-12, FP32 1e-5 relative max-norm.
"""
import numpy as np
import pytest

import seeded_inputs
from oracle import problems, spectral, stepper

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


@pytest.mark.parametrize("N,dtype,stages,bc", [
    pytest.param([11, 13], "f64", 2, "dirichlet", id="2d-11x13-f64"),
    pytest.param([22, 17], "f32", 2, "dirichlet", id="2d-22x17-f32"),
    pytest.param([11, 6, 34], "f64", 1, "dirichlet", id="3d-11x6x34-f64-eife1"),
    pytest.param([143, 8], "f64", 2, "dirichlet", id="2d-two-primes-143x8-f64"),
    pytest.param([1021, 8], "f64", 2, "dirichlet", id="2d-prime-1021x8-f64"),
    pytest.param([509, 10], "f32", 2, "dirichlet", id="2d-prime-509x10-f32"),
    pytest.param([22, 26], "f64", 2, "periodic", id="periodic-22x26-f64"),
    pytest.param([12, 11, 13], "f64", 2, "periodic", id="periodic-3d-12x11x13-f64"),
])
def test_prime_factors_above_seven(N, dtype, stages, bc):
    import paper_2209_11922_amd as eife
    h = [1.0 / n for n in N]
    D = 0.02 ** 2 if bc == "dirichlet" else 1e-3
    per = bc == "periodic"
    shape = [n if per else n - 1 for n in N]
    u0 = np.random.default_rng(31).uniform(-0.9, 0.9, tuple(reversed(shape))) if per else \
        seeded_inputs.uniform_field(31, N)
    print(f"general N {N} {dtype} EIFE{stages} {bc}", flush=True)
    g = eife.Grid(N, h, D, dtype, bc=eife.BC_PERIODIC if per else eife.BC_DIRICHLET)
    g.set_phi(0.01, stages)
    u = torch.tensor(u0, dtype=g.torch_dtype, device="cuda")
    g.step(u, 3, eife.F_ALLEN_CAHN)
    torch.cuda.synchronize()
    got = u.double().cpu().numpy()
    g.close()
    if per:
        basis = spectral.make_basis("C", N, h, D, bc="periodic")
    else:
        basis = spectral.SineBasis(N, h, D)
    ref = stepper.run(basis, u0, problems.allen_cahn(), 0.01, 3, stages)
    err = _rel(got, ref)
    print(f"  rel err {err:.2e}")
    assert err <= TOL[dtype]
