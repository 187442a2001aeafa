"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle.

Tolerances (relative max-norm of the nodal difference, floor 1e-300):
FP64 1e-12 and FP32 1e-5.  Inputs come from seeded_inputs; the oracle uses
the per-axis eigendecomposition (tier B) where it is fast enough and the
library sine transform (tier C, pinned to tiers A/B) on the large grids.
"""
import numpy as np
import pytest

import seeded_inputs
from oracle import fem, norms, problems, spectral, stepper

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _lib():
    import paper_2209_11922_amd as eife
    return eife


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _gpu_run(N, h, D, u0, tau, steps, stages, fkind, dtype="f64", c2=0.5, load=0, origin=None, t0=0.0,
             forcing=None):
    eife = _lib()
    g = eife.Grid(N, h, D, dtype)
    if c2 != 0.5:
        g.set_c2(c2)
    g.set_load(load)
    if origin is not None:
        g.set_origin(origin)
    if forcing is not None:
        g.set_forcing(*forcing)
    g.set_phi(tau, stages)
    u = torch.tensor(np.ascontiguousarray(u0), dtype=g.torch_dtype, device="cuda")
    g.step(u, steps, fkind, t0)
    torch.cuda.synchronize()
    out = u.double().cpu().numpy()
    g.close()
    return out


def _oracle(tier, N, h, D, u0, f, tau, steps, stages, c2=0.5, load="lumped", origin=None, t0=0.0):
    b = spectral.make_basis(tier, N, h, D)
    return stepper.run(b, u0, f, tau, steps, stages, c2, t0=t0, load=load, origin=origin)


def _case(name, *a, **k):
    return pytest.param(*a, id=name, **k)


AC_CASES = [
    # name, N, stages, dtype, load
    _case("cfg1-63x63-f64-eife2", [64, 64], 2, "f64", "lumped"),
    _case("63x63-f64-eife1", [64, 64], 1, "f64", "lumped"),
    _case("63x63-f64-eife2-nodal", [64, 64], 2, "f64", "nodal"),
    _case("ragged-2d-f64", [24, 9], 2, "f64", "lumped"),
    _case("ragged-2d-odd-rows-f64", [48, 8], 2, "f64", "lumped"),
    _case("1d-f64", [96], 2, "f64", "lumped"),
    _case("1d-f64-eife1", [36], 1, "f64", "nodal"),
    _case("3d-mixed-radix-f64", [16, 12, 18], 2, "f64", "lumped"),
    _case("3d-f64-eife1-nodal", [8, 16, 6], 1, "f64", "nodal"),
    _case("cfg1-63x63-f32-eife2", [64, 64], 2, "f32", "lumped"),
    _case("3d-f32", [32, 24, 16], 2, "f32", "lumped"),
    _case("tiny-2x2-f64", [2, 2], 2, "f64", "lumped"),
    _case("2x3x2-f64", [2, 3, 2], 2, "f64", "nodal"),
]


@pytest.mark.parametrize("N,stages,dtype,load", AC_CASES)
def test_allen_cahn_parity(N, stages, dtype, load):
    d = len(N)
    h = [1.0 / n for n in N]
    eps = 0.05
    u0 = seeded_inputs.uniform_field(7 + d, N)
    steps = 100 if N == [64, 64] else 25
    tau = 0.01
    got = _gpu_run(N, h, eps * eps, u0, tau, steps, stages, 1, dtype, load=0 if load == "lumped" else 1)
    ref = _oracle("B", N, h, eps * eps, u0, problems.allen_cahn(), tau, steps, stages, load=load)
    err = _rel(got, ref)
    print(f"{N} {dtype} stages={stages} load={load}: rel err {err:.3e}")
    assert err <= TOL[dtype]


def test_nonuniform_h_and_large_step():
    N, h, D = [32, 16], [0.013, 0.07], 0.9
    u0 = seeded_inputs.uniform_field(21, N)
    got = _gpu_run(N, h, D, u0, 0.37, 20, 2, 1)
    ref = _oracle("B", N, h, D, u0, problems.allen_cahn(), 0.37, 20, 2)
    assert _rel(got, ref) <= 1e-12


@pytest.mark.parametrize("c2", [1.0, 0.3])
def test_c2_variants(c2):
    N = [24, 32]
    h = [1 / 24, 1 / 32]
    u0 = seeded_inputs.uniform_field(5, N)
    got = _gpu_run(N, h, 0.01, u0, 0.02, 30, 2, 1, c2=c2)
    ref = _oracle("B", N, h, 0.01, u0, problems.allen_cahn(), 0.02, 30, 2, c2=c2)
    assert _rel(got, ref) <= 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_manufactured_problem(dtype):
    N = [64, 64]
    h = [1 / 64, 1 / 64]
    X = fem.mesh(N, h)
    u0 = problems.mms_u2_exact(0.0, X)
    got = _gpu_run(N, h, 1.0, u0, 2.0 ** -6, 64, 2, 2, dtype, t0=0.0)
    ref = _oracle("B", N, h, 1.0, u0, problems.mms_u2(1.0), 2.0 ** -6, 64, 2)
    assert _rel(got, ref) <= TOL[dtype]


def test_manufactured_problem_3d_eife1_with_time_offset():
    N = [12, 16, 8]
    h = [1 / 12, 1 / 16, 1 / 8]
    X = fem.mesh(N, h)
    u0 = problems.mms_u2_exact(0.25, X)
    got = _gpu_run(N, h, 0.5, u0, 0.01, 40, 1, 2, t0=0.25)
    ref = _oracle("B", N, h, 0.5, u0, problems.mms_u2(0.5), 0.01, 40, 1, t0=0.25)
    assert _rel(got, ref) <= 1e-12


def test_example_5_1_with_origin():
    N = [64, 32]
    h = [2 / 64, 1 / 32]
    X = fem.mesh(N, h, problems.EX51_ORIGIN)
    u0 = problems.ex51_exact(0.0, X)
    got = _gpu_run(N, h, problems.EX51_D, u0, 1 / 64, 64, 2, 3, origin=problems.EX51_ORIGIN)
    ref = _oracle("B", N, h, problems.EX51_D, u0, problems.ex51(), 1 / 64, 64, 2, origin=problems.EX51_ORIGIN)
    assert _rel(got, ref) <= 1e-12
    # and the run lands on the exact solution to within the scheme's error (Table 2 scale)
    err = norms.discrete_norms(N, h, problems.ex51_exact(1.0, X) - got)[0]
    assert err < 1e-4


@pytest.mark.parametrize("stages", [1, 2])
def test_constant_and_affine_forcing(stages):
    N = [16, 8, 12]
    h = [1 / 16, 1 / 8, 1 / 12]
    u0 = seeded_inputs.uniform_field(2, N)
    got = _gpu_run(N, h, 0.7, u0, 0.05, 7, stages, 4, forcing=(1.3, 0.0))
    ref = _oracle("B", N, h, 0.7, u0, problems.constant(1.3), 0.05, 7, stages)
    assert _rel(got, ref) <= 1e-12
    got = _gpu_run(N, h, 0.7, u0, 0.05, 7, stages, 5, forcing=(0.4, -2.0), t0=0.3)
    ref = _oracle("B", N, h, 0.7, u0, problems.affine_t(0.4, -2.0), 0.05, 7, stages, t0=0.3)
    assert _rel(got, ref) <= 1e-12


def test_single_mode_exact_decay():
    N = [32, 16]
    h = [1 / 32, 1 / 16]
    X = fem.mesh(N, h)
    u0 = np.sin(3 * np.pi * X[0]) * np.sin(2 * np.pi * X[1])
    D, tau, n = 0.2, 0.03, 11
    got = _gpu_run(N, h, D, u0, tau, n, 2, 0)
    lam = 0.0
    for a, k in enumerate([3, 2]):
        c = np.cos(k * np.pi / N[a])
        lam += 6 * (1 - c) / (h[a] ** 2 * (2 + c))
    ref = np.exp(-n * tau * D * lam) * u0
    assert _rel(got, ref) <= 1e-12


def test_zero_steps_leaves_u_untouched():
    eife = _lib()
    g = eife.Grid([16, 16], [1 / 16, 1 / 16], 1.0, "f64")
    g.set_phi(0.1, 2)
    u0 = torch.tensor(seeded_inputs.uniform_field(1, [16, 16]), device="cuda")
    u = u0.clone()
    g.step(u, 0, 1)
    torch.cuda.synchronize()
    assert torch.equal(u, u0)


def test_norms_match_oracle():
    eife = _lib()
    N = [24, 16, 12]
    h = [1 / 24, 1 / 16, 1 / 12]
    D = 0.04
    g = eife.Grid(N, h, D, "f64")
    a = seeded_inputs.uniform_field(3, N)
    b = seeded_inputs.uniform_field(4, N)
    ta = torch.tensor(a, device="cuda")
    tb = torch.tensor(b, device="cuda")
    l2, h1, mx, en = g.norms(ta, tb)
    rl2, rh1, rmx = norms.discrete_norms(N, h, a - b)
    assert l2 == pytest.approx(rl2, rel=1e-12)
    assert h1 == pytest.approx(rh1, rel=1e-12)
    assert mx == pytest.approx(rmx, rel=1e-15)
    assert en == pytest.approx(norms.allen_cahn_energy(N, h, D, a), rel=1e-12)
    l2u = g.norms(ta)[0]
    assert l2u == pytest.approx(norms.discrete_norms(N, h, a)[0], rel=1e-12)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_norms_match_oracle_across_z_chunks(dtype):
    """A 3D grid whose norm reduction marches over chunks of two z planes per thread."""
    eife = _lib()
    N = [256, 64, 24]
    h = [1 / 256, 1 / 64, 1 / 24]
    g = eife.Grid(N, h, 0.01, dtype)
    a = seeded_inputs.uniform_field(5, N)
    b = seeded_inputs.uniform_field(6, N)
    ta = torch.tensor(a, dtype=g.torch_dtype, device="cuda")
    tb = torch.tensor(b, dtype=g.torch_dtype, device="cuda")
    a64, b64 = ta.double().cpu().numpy(), tb.double().cpu().numpy()
    l2, h1, mx, en = g.norms(ta, tb)
    g.close()
    rl2, rh1, rmx = norms.discrete_norms(N, h, a64 - b64)
    assert l2 == pytest.approx(rl2, rel=1e-12)
    assert h1 == pytest.approx(rh1, rel=1e-12)
    assert mx == pytest.approx(rmx, rel=1e-15)
    assert en == pytest.approx(norms.allen_cahn_energy(N, h, 0.01, a64), rel=1e-12)


@pytest.mark.parametrize("N,dtype", [([256, 48, 36], "f32"), ([256, 48, 36], "f64"), ([64, 9, 2], "f64"),
                                     ([384, 12, 8], "f32")])
def test_norms_row_tiles_and_fallback(N, dtype):
    """3D norms with full-row tiles (rows of at most 256 nodes; a partial last row tile,
    an odd z count, a single z plane) and the column-tile reduction for longer rows."""
    eife = _lib()
    h = [1.0 / n for n in N]
    D = 0.013
    g = eife.Grid(N, h, D, dtype)
    a = seeded_inputs.uniform_field(15, N)
    b = seeded_inputs.uniform_field(16, N)
    ta = torch.tensor(a, dtype=g.torch_dtype, device="cuda")
    tb = torch.tensor(b, dtype=g.torch_dtype, device="cuda")
    a64, b64 = ta.double().cpu().numpy(), tb.double().cpu().numpy()
    l2, h1, mx, en = g.norms(ta, tb)
    l2u = g.norms(ta)[0]
    g.close()
    rl2, rh1, rmx = norms.discrete_norms(N, h, a64 - b64)
    assert l2 == pytest.approx(rl2, rel=1e-12)
    assert h1 == pytest.approx(rh1, rel=1e-12)
    assert mx == pytest.approx(rmx, rel=1e-15)
    assert en == pytest.approx(norms.allen_cahn_energy(N, h, D, a64), rel=1e-12)
    assert l2u == pytest.approx(norms.discrete_norms(N, h, a64)[0], rel=1e-12)


def test_runs_on_a_side_stream():
    eife = _lib()
    N = [64, 64]
    h = [1 / 64, 1 / 64]
    u0 = seeded_inputs.uniform_field(9, N)
    g = eife.Grid(N, h, 0.0025, "f64")
    g.set_phi(0.01, 2)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        u = torch.tensor(u0, device="cuda")
        g.step(u, 20, 1, stream=s)
    s.synchronize()
    ref = _oracle("B", N, h, 0.0025, u0, problems.allen_cahn(), 0.01, 20, 2)
    assert _rel(u.cpu().numpy(), ref) <= 1e-12


def test_abi_errors():
    eife = _lib()
    with pytest.raises(eife.EIFEError) as e:
        eife.Grid([4097, 8], [0.1, 0.1], 1.0)  # more than 4096 intervals
    assert e.value.code == -3
    with pytest.raises(eife.EIFEError) as e:
        eife.Grid([8, 8], [0.1, -0.1], 1.0)
    assert e.value.code == -1
    with pytest.raises(eife.EIFEError) as e:
        eife.Grid([8, 8], [0.1, 0.1], 1.0, bc=7)  # no such boundary condition
    assert e.value.code == -1
    with pytest.raises(eife.EIFEError) as e:
        eife.Grid([8, 1], [0.1, 0.1], 1.0, bc=eife.BC_PERIODIC)  # fewer than 2 intervals
    assert e.value.code == -1
    g = eife.Grid([8, 8], [0.1, 0.1], 1.0)
    u = torch.zeros(7, 7, dtype=torch.float64, device="cuda")
    with pytest.raises(eife.EIFEError) as e:
        g.step(u, 1, 1)
    assert e.value.code == -4
    with pytest.raises(eife.EIFEError):
        g.set_phi(-1.0, 2)
    with pytest.raises(eife.EIFEError):
        g.set_phi(0.1, 4)
    with pytest.raises(eife.EIFEError):
        g.set_c2(0.0)
    g.set_phi(0.1, 2)
    with pytest.raises(eife.EIFEError) as e:
        g.step(u, 1, 42)
    assert e.value.code == -1
    with pytest.raises(TypeError):
        g.step(u.float(), 1, 1)
    g3 = eife.Grid([4, 4, 4], [0.25] * 3, 1.0)
    g3.set_phi(0.1, 1)
    with pytest.raises(eife.EIFEError) as e:
        g3.step(torch.zeros(27, dtype=torch.float64, device="cuda"), 1, 3)  # Example 5.1 is 2D
    assert e.value.code == -1
    with pytest.raises(eife.EIFEError) as e:
        eife.Grid([8192, 8], [0.1, 0.1], 1.0)
    assert e.value.code == -3


FAST_GRIDS = [
    _case("2d-64x128", [64, 128]),
    _case("2d-256x64", [256, 64]),
    _case("2d-512x128", [512, 128]),
    _case("3d-128x64x256", [128, 64, 256]),
    _case("3d-256x96x48-mixed", [256, 96, 48]),
    _case("1d-512", [512]),
    _case("2d-192x384-radix3", [192, 384]),
    _case("3d-192x64x48-radix3", [192, 64, 48]),
    # long lines (one line pair per block): x and last axis of 1024, 2048 and 4096
    # intervals, a 3D grid with a long mid axis (generic there) and a long last axis
    _case("2d-1024x24-long", [1024, 24]),
    _case("2d-12x1024-long", [12, 1024]),
    _case("2d-2048x16-long", [2048, 16]),
    _case("2d-24x4096-long", [24, 4096]),
    _case("3d-4096x6x8-long", [4096, 6, 8]),
    _case("3d-12x8x2048-long", [12, 8, 2048]),
]


@pytest.mark.parametrize("N", FAST_GRIDS)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("stages", [1, 2])
def test_specialised_passes_match_generic_and_oracle(N, dtype, stages):
    """The specialised power-of-two passes agree with the generic passes and the oracle."""
    eife = _lib()
    h = [1.0 / n for n in N]
    D = 1e-3
    u0 = seeded_inputs.uniform_field(31, N)
    outs = []
    for tx in (eife.binding.TX_FFT, eife.binding.TX_FFT_GENERIC):
        g = eife.Grid(N, h, D, dtype)
        g.set_transform(tx)
        g.set_phi(0.01, stages)
        u = torch.tensor(u0, dtype=g.torch_dtype, device="cuda")
        g.step(u, 6, eife.F_ALLEN_CAHN)
        torch.cuda.synchronize()
        outs.append(u.double().cpu().numpy())
        g.close()
    ref = _oracle("C", N, h, D, u0, problems.allen_cahn(), 0.01, 6, stages)
    assert _rel(outs[0], ref) <= TOL[dtype]
    assert _rel(outs[1], ref) <= TOL[dtype]
    assert _rel(outs[0], outs[1]) <= TOL[dtype]


SMOOTH_GRIDS = [
    _case("1d-35", [35]),                  # 2N = 70 = 2 5 7
    _case("2d-10x14", [10, 14]),           # radix 5 and radix 7 stages
    _case("2d-100x49", [100, 49]),         # 2N = 200 = 8 25, 98 = 2 49
    _case("3d-20x21x25", [20, 21, 25]),    # 2, 3, 5 and 7 mixed
    _case("2d-1000x6", [1000, 6]),         # a long 5-smooth row
]


@pytest.mark.parametrize("N", SMOOTH_GRIDS)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_radix5_radix7_sizes_match_oracle(N, dtype):
    """Sizes whose 2N has factors 5 and 7 (generic radix-5 / radix-7 Stockham stages)
    against the oracle (scipy's DST-I: any N), EIFE2, both precisions."""
    eife = _lib()
    h = [1.0 / n for n in N]
    D = 2e-3
    u0 = seeded_inputs.uniform_field(41, N)
    g = eife.Grid(N, h, D, dtype)
    g.set_phi(0.01, 2)
    u = torch.tensor(u0, dtype=g.torch_dtype, device="cuda")
    g.step(u, 5, eife.F_ALLEN_CAHN)
    torch.cuda.synchronize()
    ref = _oracle("C", N, h, D, u0, problems.allen_cahn(), 0.01, 5, 2)
    err = _rel(u.double().cpu().numpy(), ref)
    print(f"{N} {dtype}: {err:.2e}")
    assert err <= TOL[dtype]
    g.close()


@pytest.mark.parametrize("N", [[25, 35], [20, 14, 10]])
def test_radix5_radix7_periodic_match_oracle(N):
    """Periodic grids of 5- and 7-smooth sizes (FFT length N) against the oracle."""
    eife = _lib()
    h = [1.0 / n for n in N]
    D = 1e-3
    u0 = seeded_inputs.uniform_field(42, [n + 1 for n in N])  # N nodes per axis
    g = eife.Grid(N, h, D, "f64", bc=eife.BC_PERIODIC)
    g.set_phi(0.01, 2)
    u = torch.tensor(u0, device="cuda")
    g.step(u, 5, eife.F_ALLEN_CAHN)
    torch.cuda.synchronize()
    basis = spectral.make_basis("C", N, h, D, bc="periodic")
    ref = stepper.run(basis, u0, problems.allen_cahn(), 0.01, 5, 2)
    assert _rel(u.cpu().numpy(), ref) <= 1e-12
    g.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_repeated_runs_are_bitwise_identical(dtype):
    """A grid's result depends only on its inputs, not on what it computed before."""
    eife = _lib()
    for N in ([64, 48], [96, 128], [24, 16, 64]):
        h = [1.0 / n for n in N]
        g = eife.Grid(N, h, 1e-3, dtype)
        g.set_phi(0.01, 2)
        u0 = torch.tensor(seeded_inputs.uniform_field(77, N), dtype=g.torch_dtype, device="cuda")
        outs = []
        for _ in range(3):
            u = u0.clone()
            g.step(u, 6, eife.F_ALLEN_CAHN)
            torch.cuda.synchronize()
            outs.append(u)
        assert torch.equal(outs[0], outs[1]) and torch.equal(outs[1], outs[2]), N
        g.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_step_out_equals_in_place_step(dtype):
    """eife_step_out gives eife_step's result bit for bit in the output buffer and leaves
    the input as it was; zero steps copy; input and output may be the same buffer."""
    eife = _lib()
    for N, bc in (([64, 48], eife.BC_DIRICHLET), ([512, 512], eife.BC_DIRICHLET), ([24, 16, 64], eife.BC_DIRICHLET),
                  ([32, 64], eife.BC_PERIODIC)):
        h = [1.0 / n for n in N]
        g = eife.Grid(N, h, 1e-3, dtype, bc=bc)
        g.set_phi(0.01, 2)
        shape = [n + 1 for n in N] if bc == eife.BC_PERIODIC else N  # periodic: N nodes per axis
        u0 = torch.tensor(seeded_inputs.uniform_field(78, shape), dtype=g.torch_dtype, device="cuda")
        ref = u0.clone()
        g.step(ref, 3, eife.F_ALLEN_CAHN, 0.25)
        src = u0.clone()
        dst = torch.full_like(u0, float("nan"))
        g.step_out(src, dst, 3, eife.F_ALLEN_CAHN, 0.25)
        same = u0.clone()
        g.step_out(same, same, 3, eife.F_ALLEN_CAHN, 0.25)
        zero = torch.zeros_like(u0)
        g.step_out(src, zero, 0, eife.F_ALLEN_CAHN)
        torch.cuda.synchronize()
        assert torch.equal(dst, ref) and torch.equal(same, ref), (N, bc)
        assert torch.equal(src, u0) and torch.equal(zero, u0), (N, bc)
        with pytest.raises(eife.EIFEError):
            g.step_out(src, dst, -1, eife.F_ALLEN_CAHN)
        g.close()
