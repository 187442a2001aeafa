"""eife_norms_noalloc (the entry point that allocates nothing) against eife_norms.

Two calls in a row, the second on a smaller grid, each compared with the
allocating entry point's host values at the FP64 parity bound (1e-12
relative).  Runs alone in a fresh process and after the other tests.
"""
import numpy as np
import pytest

import seeded_inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _grid(eife, N, dtype):
    h = [1.0 / n for n in N]
    g = eife.Grid(N, h, 0.02 ** 2, dtype)
    g.set_phi(0.005, 2)
    return g


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_norms_equal_allocating_norms(dtype):
    import paper_2209_11922_amd as eife
    tdt = torch.float32 if dtype == "f32" else torch.float64
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    # first a large 3D grid (the z-marching reduction), then a smaller 3D grid, then a 2D grid
    for k, N in enumerate(([128, 96, 64], [48, 32, 24], [64, 48])):
        print(f"case {k}: N={N} dtype={dtype}", flush=True)
        g = _grid(eife, N, dtype)
        u = torch.tensor(seeded_inputs.uniform_field(40 + k, N), dtype=tdt, device="cuda")
        g.step(u, 3, eife.F_ALLEN_CAHN, 0.0)
        ref = torch.tensor(seeded_inputs.uniform_field(50 + k, N), dtype=tdt, device="cuda") * 0.1 + u
        want = np.array(g.norms(u, ref))
        got = g.norms_noalloc(u, ref, out=out)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        print(f"  allocating {want}, no-alloc {got}")
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)
        # without a reference array (e = u)
        want0 = np.array(g.norms(u))
        got0 = g.norms_noalloc(u, out=out)
        torch.cuda.synchronize()
        np.testing.assert_allclose(got0.cpu().numpy(), want0, rtol=1e-12, atol=0)
        g.close()


def test_noalloc_argument_errors():
    import paper_2209_11922_amd as eife
    g = _grid(eife, [16, 16], "f32")
    u = torch.zeros(15, 15, device="cuda")
    with pytest.raises(ValueError):
        g.norms_noalloc(u, out=torch.zeros(4, dtype=torch.float32, device="cuda"))
    code = g._lib.eife_norms_noalloc(g._g, None, None, None, None)
    assert code == eife.binding.EINVAL
    g.close()
