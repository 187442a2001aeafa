"""Split-BF16 matrix-core transform (EIFE_TX_GEMM_SPLITBF16) against the FP64 oracle.

The transform is exact up to BF16-split rounding, about 2^-17 relative per
product, so the step matches the oracle to a few 1e-5 instead of FP32
round-off.  The error is printed and bounded by GEMM_TOL (a bug in the
product layout or the fused stages shows as an O(1) error); the FFT path of
the same FP32 grid is run beside it for comparison.
"""
import numpy as np
import pytest

import seeded_inputs
from oracle import fem, problems, spectral, stepper

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

GEMM_TOL = 2e-4


def _lib():
    import paper_2209_11922_amd as eife
    return eife


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _run(N, D, u0, tau, steps, stages, fkind, tx, t0=0.0, origin=None):
    eife = _lib()
    g = eife.Grid(N, [1.0 / n for n in N], D, "f32")
    g.set_transform(tx)
    if origin is not None:
        g.set_origin(origin)
    g.set_phi(tau, stages)
    u = torch.tensor(np.ascontiguousarray(u0), dtype=torch.float32, device="cuda")
    g.step(u, steps, fkind, t0)
    torch.cuda.synchronize()
    out = u.double().cpu().numpy()
    g.close()
    return out


GRIDS = [
    pytest.param([64, 64], id="2d-63x63-kp64"),
    pytest.param([96, 48], id="2d-95x47-kp128x64"),
    pytest.param([256, 256], id="2d-255x255-kp256"),
    pytest.param([512, 128], id="2d-511x127-kp512"),
    pytest.param([1024, 16], id="2d-1023x15-kp1024"),
    pytest.param([24, 36, 18], id="3d-ragged"),
    pytest.param([64, 32, 128], id="3d-63x31x127"),
    pytest.param([96], id="1d-95"),
]


@pytest.mark.parametrize("N", GRIDS)
@pytest.mark.parametrize("stages", [1, 2])
def test_gemm_transform_against_oracle(N, stages):
    eife = _lib()
    D = 1e-3
    u0 = seeded_inputs.uniform_field(41, N)
    h = [1.0 / n for n in N]
    ref = stepper.run(spectral.make_basis("C", N, h, D), u0, problems.allen_cahn(), 0.01, 6, stages)
    gemm = _run(N, D, u0, 0.01, 6, stages, eife.F_ALLEN_CAHN, eife.binding.TX_GEMM_SPLITBF16)
    fft = _run(N, D, u0, 0.01, 6, stages, eife.F_ALLEN_CAHN, eife.binding.TX_FFT)
    e_gemm, e_fft = _rel(gemm, ref), _rel(fft, ref)
    print(f"N={N} stages={stages}: split-BF16 GEMM rel max err {e_gemm:.3e}, FP32 FFT {e_fft:.3e}")
    assert e_fft <= 1e-5
    assert e_gemm <= GEMM_TOL


def test_gemm_transform_manufactured_forcing():
    """The general reaction path (space-time forcing of the manufactured problem) on the GEMM transform."""
    eife = _lib()
    N = [128, 128]
    D = 0.01
    h = [1.0 / n for n in N]
    X = fem.mesh(N, h)
    u0 = problems.mms_u2_exact(0.0, X)
    ref = stepper.run(spectral.make_basis("C", N, h, D), u0, problems.mms_u2(D), 0.02, 5, 2)
    got = _run(N, D, u0, 0.02, 5, 2, eife.F_MMS_U2, eife.binding.TX_GEMM_SPLITBF16)
    e = _rel(got, ref)
    print(f"MMS 127^2 split-BF16 GEMM rel max err {e:.3e}")
    assert e <= GEMM_TOL


def test_gemm_transform_255_cubed():
    """The 3D Allen-Cahn workload (255^3, eps = 0.02, tau = 0.005): GEMM and FFT vs the FP64 oracle."""
    eife = _lib()
    N = [256] * 3
    D = 4e-4
    u0 = seeded_inputs.uniform_field(0, N)
    h = [1.0 / 256] * 3
    ref = stepper.run(spectral.SineBasis(N, h, D), u0, problems.allen_cahn(), 0.005, 3, 2)
    gemm = _run(N, D, u0, 0.005, 3, 2, eife.F_ALLEN_CAHN, eife.binding.TX_GEMM_SPLITBF16)
    fft = _run(N, D, u0, 0.005, 3, 2, eife.F_ALLEN_CAHN, eife.binding.TX_FFT)
    e_gemm, e_fft = _rel(gemm, ref), _rel(fft, ref)
    print(f"255^3 3 steps: split-BF16 GEMM rel max err {e_gemm:.3e}, FP32 FFT {e_fft:.3e}")
    assert e_fft <= 1e-5
    assert e_gemm <= GEMM_TOL


def test_gemm_transform_is_deterministic_and_switchable():
    eife = _lib()
    N = [128, 96]
    g = eife.Grid(N, [1.0 / n for n in N], 1e-3, "f32")
    g.set_phi(0.01, 2)
    u0 = torch.tensor(seeded_inputs.uniform_field(5, N), dtype=torch.float32, device="cuda")
    outs = {}
    for tx in (eife.binding.TX_GEMM_SPLITBF16, eife.binding.TX_FFT, eife.binding.TX_GEMM_SPLITBF16):
        g.set_transform(tx)
        u = u0.clone()
        g.step(u, 4, eife.F_ALLEN_CAHN)
        torch.cuda.synchronize()
        if tx in outs:
            assert torch.equal(outs[tx], u)
        outs[tx] = u
    assert not torch.equal(outs[eife.binding.TX_FFT], outs[eife.binding.TX_GEMM_SPLITBF16])
    g.close()


def test_gemm_transform_rejections():
    eife = _lib()
    g = eife.Grid([64, 64], [1 / 64] * 2, 1e-3, "f64")
    with pytest.raises(eife.EIFEError) as e:
        g.set_transform(eife.binding.TX_GEMM_SPLITBF16)
    assert e.value.code == -3
    g.close()
    g = eife.Grid([1536, 8], [1 / 1536, 1 / 8], 1e-3, "f32")
    with pytest.raises(eife.EIFEError) as e:
        g.set_transform(eife.binding.TX_GEMM_SPLITBF16)
    assert e.value.code == -3
    with pytest.raises(eife.EIFEError) as e:
        g.set_transform(7)
    assert e.value.code == -1
    g.close()
