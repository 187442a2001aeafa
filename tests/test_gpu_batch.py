"""Batched instances (one launch per size class per pass, HIP-graph replay, autotuned shapes).

Each instance of a batch must reproduce, bit for bit, a single grid of the
same size: both run the same kernels and the per-line arithmetic does not
depend on the launch shape.  A sample is also checked against the oracle.
"""
import json

import numpy as np
import pytest

import seeded_inputs
from oracle import problems, spectral, stepper

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _eife():
    import paper_2209_11922_amd as eife
    return eife


def _mixed_instances():
    # (Nx, Ny, D): power-of-two and radix-3 sizes, repeated sizes, rectangular grids
    return [(64, 64, 0.0025), (96, 96, 1e-3), (128, 128, 4e-4), (48, 48, 2e-3), (64, 64, 9e-4),
            (128, 64, 1e-3), (128, 128, 2.5e-3), (24, 36, 5e-3)]


def _inputs(inst, seed0=100):
    return [seeded_inputs.uniform_field(seed0 + i, [nx, ny]) for i, (nx, ny, _) in enumerate(inst)]


def _single(nx, ny, D, u0, tau, steps, stages, dtype):
    eife = _eife()
    g = eife.Grid([nx, ny], [1.0 / nx, 1.0 / ny], D, dtype)
    g.set_phi(tau, stages)
    u = torch.tensor(u0, dtype=g.torch_dtype, device="cuda")
    g.step(u, steps, eife.F_ALLEN_CAHN)
    torch.cuda.synchronize()
    out = u.cpu().numpy()
    g.close()
    return out


def _batch_run(inst, u0s, tau, steps, stages, dtype, autotune=None, graph=True):
    eife = _eife()
    b = eife.Batch([(nx, ny, 1.0 / nx, 1.0 / ny, D) for nx, ny, D in inst], dtype)
    b.set_phi(tau, stages)
    if autotune is not None:
        b.autotune(autotune)
    u = torch.cat([torch.tensor(x.reshape(-1), dtype=b.torch_dtype) for x in u0s]).cuda()
    b.step(u, steps, eife.F_ALLEN_CAHN, graph=graph)
    torch.cuda.synchronize()
    outs = [v.cpu().numpy() for v in b.views(u)]
    return b, outs


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("stages", [1, 2])
def test_batch_equals_single_grids_bitwise(dtype, stages):
    inst = _mixed_instances()
    u0s = _inputs(inst)
    b, outs = _batch_run(inst, u0s, 0.01, 7, stages, dtype)
    assert len(b.class_info()) == 6
    for (nx, ny, D), u0, got in zip(inst, u0s, outs):
        ref = _single(nx, ny, D, u0, 0.01, 7, stages, dtype)
        assert np.array_equal(got, ref), (nx, ny)
    b.close()


@pytest.mark.parametrize("stages", [1, 2])
def test_batch_long_column_classes_equal_single_grids_bitwise(stages):
    """FP32 classes of 1024-point columns (512 intervals) run the pipelined stage pass
    over every tile of every instance (768-point columns the one-tile form); each
    instance equals its single grid (one tile per block) bit for bit."""
    inst = [(512, 512, 4e-4), (512, 512, 2.5e-3), (512, 512, 1e-4), (384, 384, 9e-4), (384, 384, 1.6e-3),
            (256, 512, 1e-3)]
    u0s = _inputs(inst, 300)
    b, outs = _batch_run(inst, u0s, 0.01, 4, stages, "f32")
    for (nx, ny, D), u0, got in zip(inst, u0s, outs):
        ref = _single(nx, ny, D, u0, 0.01, 4, stages, "f32")
        assert np.array_equal(got, ref), (nx, ny, D)
    b.close()


@pytest.mark.parametrize("var_col", [0, 1, 2, 3])
def test_every_column_variant_equals_single_grids_bitwise(tmp_path, var_col):
    """Each column-pass variant of the specialised lengths (two tile widths, one
    tile per block or the persistent stage pass), forced through the tuning
    cache, gives every instance its single grid's bits."""
    inst = [(512, 512, 4e-4), (512, 512, 2.5e-3), (384, 384, 9e-4), (256, 256, 1e-3), (128, 128, 2e-3),
            (192, 192, 1.6e-3)]
    u0s = _inputs(inst, 400)
    cache = tmp_path / "tune.json"
    b0, _ = _batch_run(inst, u0s, 0.01, 1, 2, "f32", autotune=cache)
    b0.close()
    rec = json.loads(cache.read_text())
    for key, val in rec.items():
        if val[2] == 0 and val[3] == 0:  # a class of specialised lengths
            val[1] = var_col
    # the library reads one entry per line
    cache.write_text("{\n" + ",\n".join(f'  "{k}": {json.dumps(v)}' for k, v in rec.items()) + "\n}\n")
    b, outs = _batch_run(inst, u0s, 0.01, 3, 2, "f32", autotune=cache)
    assert all(info[4] == var_col for info in b.class_info())
    for (nx, ny, D), u0, got in zip(inst, u0s, outs):
        ref = _single(nx, ny, D, u0, 0.01, 3, 2, "f32")
        assert np.array_equal(got, ref), (nx, ny, D, var_col)
    b.close()


def test_autotune_ignores_invalid_cache_entries(tmp_path):
    """Cache entries naming shapes a class cannot take are ignored and the class is tuned again."""
    inst = [(128, 128, 2e-3), (96, 96, 1e-3), (40, 40, 1e-3)]
    u0s = _inputs(inst, 500)
    cache = tmp_path / "tune.json"
    b0, ref = _batch_run(inst, u0s, 0.01, 2, 2, "f32", autotune=cache)
    b0.close()
    rec = json.loads(cache.read_text())
    for key, val in rec.items():
        if val[2] == 0 and val[3] == 0:
            val[1] = 9  # no such column variant
        else:
            val[2], val[3] = 1000, 3  # too many pairs for the LDS; pairs that do not divide the pitch
    cache.write_text("{\n" + ",\n".join(f'  "{k}": {json.dumps(v)}' for k, v in rec.items()) + "\n}\n")
    b, outs = _batch_run(inst, u0s, 0.01, 2, 2, "f32", autotune=cache)
    for info in b.class_info():
        assert 0 <= info[3] <= 64 and 0 <= info[4] <= 64, info
    for a, c in zip(ref, outs):
        assert np.array_equal(a, c)
    b.close()


def test_batch_matches_oracle():
    inst = _mixed_instances()
    u0s = _inputs(inst, 7)
    b, outs = _batch_run(inst, u0s, 0.01, 10, 2, "f64")
    for (nx, ny, D), u0, got in zip(inst, u0s, outs):
        N, h = [nx, ny], [1.0 / nx, 1.0 / ny]
        ref = stepper.run(spectral.make_basis("B", N, h, D), u0, problems.allen_cahn(), 0.01, 10, 2)
        assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) <= 1e-12
    b.close()


def test_graph_replays_match_eager_each_time():
    """The cached graph is replayed three times, with eager work in between."""
    eife = _eife()
    inst = _mixed_instances()[:5]
    u0s = _inputs(inst, 50)
    b = eife.Batch([(nx, ny, 1.0 / nx, 1.0 / ny, D) for nx, ny, D in inst], "f32")
    b.set_phi(0.01, 2)
    init = torch.cat([torch.tensor(x.reshape(-1), dtype=torch.float32) for x in u0s]).cuda()
    eager = init.clone()
    b.step(eager, 5, eife.F_ALLEN_CAHN, graph=False)
    torch.cuda.synchronize()
    u = init.clone()
    s = torch.cuda.Stream()
    for rep in range(3):
        u.copy_(init)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            b.step(u, 5, eife.F_ALLEN_CAHN, stream=s)  # same arguments: replay after the first
        s.synchronize()
        assert torch.equal(u, eager), rep
        # unrelated eager work on the device between replays
        scratch = torch.randn(1 << 20, device="cuda")
        (scratch * 2).sum().item()
    b.close()


def test_autotune_writes_and_reuses_cache(tmp_path):
    inst = _mixed_instances()
    u0s = _inputs(inst, 3)
    cache = tmp_path / "tune.json"
    b1, outs1 = _batch_run(inst, u0s, 0.01, 4, 2, "f32", autotune=cache)
    rec = json.loads(cache.read_text())
    assert len(rec) == len(b1.class_info())
    for key, val in rec.items():
        assert len(val) == 5 and val[4] > 0
    b2, outs2 = _batch_run(inst, u0s, 0.01, 4, 2, "f32", autotune=cache)
    assert b1.class_info() == b2.class_info()
    for a, c in zip(outs1, outs2):
        assert np.array_equal(a, c)
    # tuned shapes change nothing numerically
    b3, outs3 = _batch_run(inst, u0s, 0.01, 4, 2, "f32")
    for a, c in zip(outs1, outs3):
        assert np.array_equal(a, c)
    for b in (b1, b2, b3):
        b.close()


def test_batched_workload_sample_against_oracle():
    """A sample of the batched workload's instances (sizes 128..512, eps in [0.01, 0.05])."""
    draws = seeded_inputs.batch_instances(0, 512)
    picked = []
    for n in (128, 192, 256, 384, 512):
        picked.append(next(d for d in draws if d[0] == n))
    inst = [(n, n, e * e) for n, e, _ in picked]
    u0s = [seeded_inputs.uniform_field(s, [n, n]) for n, _, s in picked]
    b, outs = _batch_run(inst, u0s, 0.01, 3, 2, "f32")
    for (n, _, D), u0, got in zip(inst, u0s, outs):
        ref = stepper.run(spectral.SineBasis([n, n], [1.0 / n] * 2, D), u0, problems.allen_cahn(), 0.01, 3, 2)
        assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) <= 1e-5, n
    b.close()
