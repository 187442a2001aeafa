"""Throughput benchmark of the EIFE hot path on one MI355X.

Workload: 3D Allen-Cahn u_t = eps^2 Lap u + u - u^3, eps = 0.02, on (0,1)^3 with
256^3 Q1 intervals (255^3 = 16,581,375 interior DoFs), homogeneous Dirichlet
data, u0 i.i.d. uniform[-0.9, 0.9] (seed 0), EIFE2 (c2 = 1/2) with tau = 0.005,
FP32 sine transforms with double phi factors.  A "step" is one EIFE2 time
step of the whole grid; `--steps K` steps run in one library call after
`--warmup W` untimed steps.

Prints one JSON line: DoF-steps/s, the roofline of the dominant pass kernel
(algorithmic bytes per launch / mean launch time from HIP events recorded
around every pass on the step's stream), and the CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import seeded_inputs  # noqa: E402

METRIC = "ETDRK2 DoF-steps/s plain vs learned-corrector at equal L2 error; % HBM peak"
HBM_PEAK_GBS = 8000.0

N_INT = 256
EPS = 0.02
TAU = 0.005
SEED = 0

# Algorithmic HBM bytes per interior DoF of one launch of each pass kind
# (FP32 elements; each pass reads and writes the work array once, the two
# last-axis stage passes also read and write the spectral state).
BYTES_PER_DOF = {"row_phys": 8, "mid": 8, "last_a": 16, "last_b": 16, "row_fwd": 12, "row_inv": 8,
                 "last_plain": 8}


# Sine-matrix products per launch of each pass kind on the matrix-core transform.
GEMMS_PER_PASS = {"row_phys": 2, "mid": 1, "last_a": 2, "last_b": 2, "row_fwd": 1, "row_inv": 1, "last_plain": 1}
BF16_PEAK_TFS = 2500.0


def measured_traffic(pass_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None.

    The record is only used while the kernel sources are byte-identical to the
    ones the counters were taken on (sha256 over the two kernel headers).
    """
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", "traffic_255cubed_f32.json")
    csrc = os.path.join(ROOT, "paper_2209_11922_amd", "csrc")
    try:
        rec = json.load(open(rec_path))
        src = open(os.path.join(csrc, "eife_fast.hpp"), "rb").read() + \
            open(os.path.join(csrc, "eife_kernels.hpp"), "rb").read()
    except OSError:
        return None
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return rec.get("bytes_per_launch", {}).get(pass_name)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(u0, N, h, D, budget_s=15.0, max_steps=20):
    """Time the FP64 CPU oracle (tier C) on the first steps of the same problem."""
    from oracle import problems, spectral, stepper
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    basis = spectral.SineBasis(N, h, D, workers=cores)
    t0 = time.perf_counter()
    U = stepper.run(basis, u0, problems.allen_cahn(), TAU, 1, 2)
    one = time.perf_counter() - t0
    steps = int(max(1, min(max_steps, budget_s // max(one, 1e-3))))
    t0 = time.perf_counter()
    stepper.run(basis, U, problems.allen_cahn(), TAU, steps, 2, t0=TAU)
    dt = time.perf_counter() - t0
    ndof = int(np.prod([n - 1 for n in N]))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": ndof * steps / dt, "unit": "DoF-steps/s", "cores": cores, "cpu_model": model, "kind": "oracle",
            "sample": f"{steps} EIFE2 steps of the same 255^3 problem (after 1 untimed step), FP64 oracle tier C "
                      f"(scipy.fft.dstn type-I, workers={cores}), {dt:.2f} s"}


SETTLE_S = 1.0  # untimed stepping before the warm-up steps: the GPU's clocks ramp over tens of ms of load


def settle(torch, g, u, f_kind, seconds=SETTLE_S, chunk=50):
    """Step a scratch copy of u for about `seconds` (untimed, result discarded) so that the
    timed steps run at the device's steady clock; a 20-step run without it measures the
    ramp (per-pass times about 12% above their steady values).  Returns the steps taken."""
    scratch = u.clone()
    taken = 0
    t0 = time.perf_counter()
    while True:
        g.step(scratch, chunk, f_kind, 0.0)
        taken += chunk
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= seconds:
            break
    del scratch
    return taken


def reduction_rate(torch, g, u, ndof, calls=10):
    """The FP64 norm and energy reduction on the benchmark grid against a second array: the
    device time per call (eife_norms_noalloc, values left in device memory, event-timed on
    the stream it runs on), the wall time of eife_norms (it returns the four values to the
    host) and the algorithmic rate, two FP32 arrays read once."""
    ref = torch.zeros_like(u)
    g.norms(u, ref)
    out = torch.empty(4, dtype=torch.float64, device=u.device)
    stream = torch.cuda.current_stream()
    g.norms_noalloc(u, ref, out, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(calls):
        g.norms_noalloc(u, ref, out, stream)
    e1.record(stream)
    e1.synchronize()
    dev = e0.elapsed_time(e1) * 1e-3 / calls
    t0 = time.perf_counter()
    for _ in range(calls):
        vals = g.norms(u, ref)
    dt = (time.perf_counter() - t0) / calls
    gbs = 2 * 4 * ndof / dev / 1e9
    log(f"bench: norms {dev * 1e6:.1f} us per call on the device, {gbs:.1f} GB/s algorithmic "
        f"({gbs / HBM_PEAK_GBS * 100:.1f}% of HBM peak); {dt * 1e6:.1f} us with the host round trip")
    del ref
    return {"us_per_call": round(dev * 1e6, 1), "us_per_call_host_round_trip": round(dt * 1e6, 1),
            "alg_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_per_call": 2 * 4 * ndof, "values": list(vals)}


def accuracy_vs_f64(torch, eife, u0, N, h, D, steps):
    """Relative max-norm error of the benchmark problem after `steps` EIFE2 steps for the FP32
    sine-transform path and the split-BF16 matrix-core path, against the FP64 sine-transform
    path (itself held to the FP64 oracle at 1e-12 by the parity tests)."""
    def run(dtype, kind):
        g = eife.Grid(N, h, D, dtype)
        if kind == "gemm":
            g.set_transform(eife.binding.TX_GEMM_SPLITBF16)
        g.set_phi(TAU, 2)
        u = torch.tensor(u0, dtype=torch.float64 if dtype == "f64" else torch.float32, device="cuda")
        g.step(u, steps, eife.F_ALLEN_CAHN, 0.0)
        torch.cuda.synchronize()
        g.close()
        return u.double()
    ref = run("f64", "fft")
    scale = float(ref.abs().max())
    out = {"steps": steps, "reference": "FP64 sine-transform path"}
    for key, dtype, kind in (("fft_f32", "f32", "fft"), ("gemm_bf16x3", "f32", "gemm")):
        out[key] = float((run(dtype, kind) - ref).abs().max()) / scale
    log(f"bench: after {steps} steps, rel max error vs FP64: FFT FP32 {out['fft_f32']:.2e}, "
        f"split-BF16 GEMM {out['gemm_bf16x3']:.2e}")
    return out


def f64_rate(torch, eife, u0, N, h, D, steps, settle_s):
    """The same 255^3 problem in FP64 (the paper's precision): event-free wall timing of
    `steps` steps after a settle and 5 warm-up steps, with the step's algorithmic HBM rate
    (every pass reads and writes FP64 arrays: twice the FP32 bytes, 160 B/DoF)."""
    g = eife.Grid(N, h, D, "f64")
    g.set_phi(TAU, 2)
    u = torch.tensor(u0, dtype=torch.float64, device="cuda")
    if settle_s > 0:
        settle(torch, g, u, eife.F_ALLEN_CAHN, min(settle_s, 0.5))
    g.step(u, 5, eife.F_ALLEN_CAHN, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(u, steps, eife.F_ALLEN_CAHN, 5 * TAU)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    g.close()
    ndof = int(np.prod([n - 1 for n in N]))
    gbs = 160 * ndof / dt / 1e9
    log(f"bench: FP64 {dt * 1e3:.3f} ms/step, {ndof / dt:.4e} DoF-steps/s, {gbs:.1f} GB/s algorithmic "
        f"({gbs / HBM_PEAK_GBS * 100:.1f}% of HBM peak)")
    return {"ms_per_step": round(dt * 1e3, 4), "dof_steps_per_s": ndof / dt, "bytes_per_dof": 160,
            "alg_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4), "steps": steps}


def corrector_comparison(nseeds):
    """Learned corrector vs plain EIFE2 at equal L2 error (2D Allen-Cahn, eps 0.02,
    511^2 DoFs, coarse tau 0.016, fine 0.002, 500 coarse steps, unseen seeds 1000...)."""
    from paper_2209_11922_amd import corrector as cor
    from paper_2209_11922_amd.binding import Corrector
    path = os.path.join(ROOT, "paper_2209_11922_amd", "weights", "corrector_ac512.npz")
    p, s_out, theta, guard = cor.load(path)
    net = Corrector(511, 511, 1)
    net.set_params(p)
    net.set_scale(s_out)
    t0 = time.perf_counter()
    summ = cor.compare(net, list(range(1000, 1000 + nseeds)), 500, theta, guard)
    net.close()
    comp = summ.get("plain_competitor")
    log(f"bench: corrector {summ['corrector']['fine_equiv_dof_steps_per_s']:.4e} fine-equivalent DoF-steps/s, "
        f"max L2 {summ['corrector']['max_L2']:.2e}; competitor {comp} "
        f"{summ[comp]['fine_equiv_dof_steps_per_s'] if comp else float('nan'):.4e}, "
        f"max L2 {summ[comp]['max_L2'] if comp else float('nan'):.2e} ({time.perf_counter() - t0:.1f} s)")
    return summ


def bench_manufactured(args, torch, eife):
    """The manufactured 2D problem u_t = Δu + u^2 + g on (0,1)^2 with exact solution
    u = e^{-t} sin(pi x) sin(pi y), 4096^2 intervals (4095^2 DoFs), T = 1, tau = 2^-4 ... 2^-10,
    EIFE1 and EIFE2, FP64 transforms and FP32 transforms with FP64 phi factors.  Per run: the
    L2/H1/max errors against the exact nodal values (time and space error, as Section 5 reports
    them) and DoF-steps/s; the temporal order is fitted on the FP64 runs against a same-grid
    FP64 reference at tau = 2^-13 (which removes the h^2 floor of the exact-solution errors)."""
    n_int = 4096
    N, h = [n_int, n_int], [1.0 / n_int] * 2
    ndof = (n_int - 1) ** 2
    s = np.sin(np.pi * np.arange(1, n_int) / n_int)
    base = np.outer(s, s)  # [y][x], x fastest
    ks = list(range(4, 11))
    k_ref = 13
    log(f"bench: manufactured 2D u^2 + g, {n_int - 1}^2 DoFs, T = 1, tau = 2^-{ks[0]} .. 2^-{ks[-1]}")

    def run(dtype, stages, k):
        tdt = torch.float64 if dtype == "f64" else torch.float32
        g = eife.Grid(N, h, 1.0, dtype)
        g.set_phi(2.0 ** -k, stages)
        u = torch.tensor(base, dtype=tdt, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(u, 2 ** k, eife.F_MMS_U2, 0.0)
        torch.cuda.synchronize()
        return g, u, time.perf_counter() - t0

    exact = {d: torch.tensor(np.exp(-1.0) * base, dtype=torch.float64 if d == "f64" else torch.float32,
                             device="cuda") for d in ("f64", "f32")}
    res = {}
    for stages in (1, 2):
        g_ref, u_ref, _ = run("f64", stages, k_ref)
        g_ref.close()
        for dtype in ("f64", "f32"):
            rows = []
            for k in ks:
                g, u, dt = run(dtype, stages, k)
                l2, h1, mx, _ = g.norms(u, exact[dtype])
                row = {"tau": 2.0 ** -k, "steps": 2 ** k, "L2_vs_exact": l2, "H1_vs_exact": h1, "max_vs_exact": mx,
                       "dof_steps_per_s": ndof * 2 ** k / dt}
                if dtype == "f64":
                    row["L2_vs_tau_ref"] = g.norms(u, u_ref)[0]
                g.close()
                rows.append(row)
            key = f"{dtype}_eife{stages}"
            res[key] = {"rows": rows}
            msg = (f"  {key}: L2 vs exact at tau=2^-{ks[-1]} {rows[-1]['L2_vs_exact']:.3e}, "
                   f"{rows[-1]['dof_steps_per_s']:.3e} DoF-steps/s")
            if dtype == "f64":
                sl = np.polyfit(np.log([r["tau"] for r in rows[-3:]]),
                                np.log([r["L2_vs_tau_ref"] for r in rows[-3:]]), 1)[0]
                res[key]["temporal_order_L2"] = round(float(sl), 3)
                res[key]["tau_ref"] = 2.0 ** -k_ref
                msg += f", temporal order {sl:.3f}"
            log(msg)
        del u_ref
    best = res["f32_eife2"]["rows"][-1]
    out = {"metric": "manufactured 2D EIFE DoF-steps/s, errors and observed temporal orders",
           "value": best["dof_steps_per_s"], "unit": "DoF-steps/s", "n_gpus": 1, "steps": best["steps"],
           "warmup": 0, "ms_per_step": 1e3 * ndof / best["dof_steps_per_s"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "manufactured 2D u_t = Δu + u^2 + g, exact e^{-t} sin(pi x) sin(pi y), "
                                  "4096^2 intervals, T = 1; value: FP32 EIFE2 at tau = 2^-10", "dofs": ndof},
           "manufactured": res}
    print(json.dumps(out), flush=True)
    return 0


def bench_ex53(args, torch, eife):
    """Example 5.3 (Section 5.2), grain coarsening: u_t = eps^2 Lap u + (theta/2) ln((1-u)/(1+u)) + theta_c u
    on the periodic unit cube, eps = 0.01, theta = 0.8, theta_c = 1.6, 128^3 intervals (128^3 DoFs),
    u0 i.i.d. uniform[-0.9, 0.9] per mesh point (seeded), EIFE2 with tau = 5/512 to T = 20 (2048 steps).
    Per dtype: the whole 2048-step run timed in one call, a second run that records max|u| and the
    discrete energy every 64 steps (maximum bound gamma ~ 0.9575 and monotone energy decay, the two
    properties Section 5.2 plots), and per-pass event timings over 64 steps."""
    n, tau, steps, every = 128, 5.0 / 512.0, 2048, 64
    theta, theta_c = 0.8, 1.6
    N, h, D = [n] * 3, [1.0 / n] * 3, 0.01 ** 2
    ndof = n ** 3
    u0 = seeded_inputs.uniform_field(SEED, [n + 1] * 3)  # n^3 periodic nodes
    # maximum bound: the positive root of the reaction (theta/2) ln((1-u)/(1+u)) + theta_c u
    lo, hi = 0.5, 1.0 - 1e-12
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if 0.5 * theta * np.log((1 - mid) / (1 + mid)) + theta_c * mid > 0 else (lo, mid)
    gamma = 0.5 * (lo + hi)
    log(f"bench: Example 5.3, periodic {n}^3 Flory-Huggins EIFE2 tau=5/512, {steps} steps to T = 20")
    res = {}
    for dtype in ("f64", "f32"):
        tdt = torch.float64 if dtype == "f64" else torch.float32
        esz = 8 if dtype == "f64" else 4
        g = eife.Grid(N, h, D, dtype, bc=eife.BC_PERIODIC)
        g.set_forcing(theta, theta_c)
        g.set_phi(tau, 2)
        u = torch.tensor(u0, dtype=tdt, device="cuda")
        g.step(u, 16, eife.F_FLORY_HUGGINS, 0.0)  # warmup
        u.copy_(torch.tensor(u0, dtype=tdt))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(u, steps, eife.F_FLORY_HUGGINS, 0.0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        u_timed = u.clone()
        # checkpointed run of the same steps: max|u| and energy every `every` steps
        u.copy_(torch.tensor(u0, dtype=tdt))
        maxima, energies = [g.norms(u)[2]], [g.energy(u, eife.F_FLORY_HUGGINS)]
        for k in range(steps // every):
            g.step(u, every, eife.F_FLORY_HUGGINS, k * every * tau)
            maxima.append(g.norms(u)[2])
            energies.append(g.energy(u, eife.F_FLORY_HUGGINS))
        # each call converts the nodal u to the spectral state and back once, so chunking
        # changes rounding only
        chunk_diff = float((u - u_timed).abs().max()) / float(u_timed.abs().max())
        dE = np.diff(energies)
        g.profile(True)
        g.step(u, every, eife.F_FLORY_HUGGINS, steps * tau)
        prof = g.profile_read()
        g.profile(False)
        torch.cuda.synchronize()
        passes = {}
        for name, (ms, cnt) in prof.items():
            if cnt:
                avg = ms / cnt
                passes[name] = {"launches": cnt, "avg_us": round(avg * 1e3, 2),
                                "alg_GBs": round(BYTES_PER_DOF[name] * esz / 4 * ndof / (avg * 1e-3) / 1e9, 1)}
        dom = max(passes.items(), key=lambda kv: kv[1]["avg_us"] * kv[1]["launches"])
        res[dtype] = {"dof_steps_per_s": ndof * steps / dt, "ms_per_step": dt * 1e3 / steps,
                      "max_abs_u": {"t0": maxima[0], "max_over_run": max(maxima), "T": maxima[-1]},
                      "maximum_bound": {"gamma": gamma, "rel_excess": (max(maxima) - gamma) / gamma,
                                        "held_to_4_digits": bool(round(max(maxima), 4) <= round(gamma, 4))},
                      "energy": {"t0": energies[0], "T": energies[-1], "checkpoints": len(energies),
                                 "increases": int(np.sum(dE > 0)), "max_increase": float(max(dE.max(), 0.0))},
                      "checkpointed_vs_timed_rel_max_diff": chunk_diff,
                      "passes": passes,
                      "roofline": {"bound": "hbm", "kernel": dom[0], "achieved": dom[1]["alg_GBs"],
                                   "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": round(dom[1]["alg_GBs"] / HBM_PEAK_GBS, 4), "traffic": None}}
        log(f"  {dtype}: {dt * 1e3 / steps:.3f} ms/step, {ndof * steps / dt:.4e} DoF-steps/s; max|u| "
            f"{maxima[-1]:.9f} (max over run {max(maxima):.9f}, gamma {gamma:.9f}); energy {energies[0]:.6f} -> "
            f"{energies[-1]:.6f}, {int(np.sum(dE > 0))} increases over {len(dE)} intervals; dominant pass "
            f"{dom[0]} {dom[1]['alg_GBs']:.1f} GB/s")
        g.close()
        del u, u_timed
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_ex53(u0, N, h, D, tau, theta, theta_c)
        log(f"bench: cpu oracle {cpu['value']:.4e} DoF-steps/s on {cpu['cores']} cores")
    best = res["f64"]
    out = {"metric": "Example 5.3 grain coarsening EIFE2 DoF-steps/s, maximum bound and energy decay",
           "value": best["dof_steps_per_s"], "unit": "DoF-steps/s", "n_gpus": 1, "steps": steps, "warmup": 16,
           "ms_per_step": best["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "Example 5.3: 3D Flory-Huggins Allen-Cahn, periodic, 128^3 intervals, eps=0.01, "
                                  "theta=0.8, theta_c=1.6, u0 uniform[-0.9,0.9] seed 0, EIFE2 tau=5/512, T=20; "
                                  "value: FP64", "dofs": ndof, "tau": tau, "scheme": "EIFE2"},
           "roofline": best["roofline"], "cpu_baseline": cpu, "ex53": res}
    print(json.dumps(out), flush=True)
    return 0


def cpu_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def cpu_oracle_rate(one_step, run_steps, ndof, budget_s, max_steps, cores, sample):
    """Time the oracle: one untimed step, then as many steps as fit the budget (at most max_steps)."""
    t0 = time.perf_counter()
    state = one_step()
    one = time.perf_counter() - t0
    steps = int(max(1, min(max_steps, budget_s // max(one, 1e-3))))
    t0 = time.perf_counter()
    run_steps(state, steps)
    dt = time.perf_counter() - t0
    return {"value": ndof * steps / dt, "unit": "DoF-steps/s", "cores": cores, "kind": "oracle",
            "sample": sample.format(steps=steps, dt=dt)}


def cpu_baseline_ex53(u0, N, h, D, tau, theta, theta_c, budget_s=12.0, max_steps=20):
    """Time the FP64 CPU oracle (periodic tier C) on the first steps of Example 5.3."""
    from oracle import problems, spectral, stepper
    basis = spectral.make_basis("C", N, h, D, bc="periodic")
    f = problems.flory_huggins(theta, theta_c)
    t0 = time.perf_counter()
    U = stepper.run(basis, u0, f, tau, 1, 2)
    one = time.perf_counter() - t0
    steps = int(max(1, min(max_steps, budget_s // max(one, 1e-3))))
    t0 = time.perf_counter()
    stepper.run(basis, U, f, tau, steps, 2, t0=tau)
    dt = time.perf_counter() - t0
    ndof = int(np.prod(N))
    return {"value": ndof * steps / dt, "unit": "DoF-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} EIFE2 steps of Example 5.3 at 128^3 (after 1 untimed step), FP64 oracle "
                      f"periodic tier C (numpy real FFTs, one thread), {dt:.2f} s"}


def q1_errors_wave(U, N, h, t, eps, npts=4, zchunk=4):
    """Continuous L2 and H1 errors of the 3D Q1 function with interior nodal values U
    (boundary nodes: the exact traveling wave) against Example 5.2's exact solution,
    npts Gauss points per axis and element, summed over slabs of zchunk element layers."""
    w2 = 2.0 * np.sqrt(2.0) * eps
    s = 3.0 / (np.sqrt(2.0) * eps)
    u_ex = lambda x: 0.5 * (1.0 - np.tanh((x - s * t) / w2))
    ux_ex = lambda x: -0.5 / w2 / np.cosh((x - s * t) / w2) ** 2
    nx, ny, nz = N
    x = h[0] * np.arange(nx + 1)
    full = np.broadcast_to(u_ex(x), (nz + 1, ny + 1, nx + 1)).copy()
    full[1:nz, 1:ny, 1:nx] = U.reshape(nz - 1, ny - 1, nx - 1)
    gq, wq = np.polynomial.legendre.leggauss(npts)
    gq, wq = (gq + 1.0) / 2.0, wq / 2.0
    xq = (x[:-1, None] + h[0] * gq[None, :]).reshape(-1)  # (cell, q) flattened
    ue, uxe = u_ex(xq), ux_ex(xq)
    wxyz = np.einsum("i,j,k->ijk", wq, wq, wq) * h[0] * h[1] * h[2]
    l2 = semi = 0.0
    for z0 in range(0, nz, zchunk):
        z1 = min(nz, z0 + zchunk)
        Fz = full[z0:z1 + 1]
        for qz, gz in enumerate(gq):
            Fzq = Fz[:-1] * (1 - gz) + Fz[1:] * gz            # value at z point
            Dz = (Fz[1:] - Fz[:-1]) / h[2]                      # z derivative
            for qy, gy in enumerate(gq):
                V = Fzq[:, :-1] * (1 - gy) + Fzq[:, 1:] * gy    # (cz, ny, nx + 1)
                Dy = (Fzq[:, 1:] - Fzq[:, :-1]) / h[1]
                Vz = Dz[:, :-1] * (1 - gy) + Dz[:, 1:] * gy
                for qx, gx in enumerate(gq):
                    w = wxyz[qx, qy, qz]
                    uh = V[..., :-1] * (1 - gx) + V[..., 1:] * gx
                    dx = (V[..., 1:] - V[..., :-1]) / h[0]
                    dy = Dy[..., :-1] * (1 - gx) + Dy[..., 1:] * gx
                    dz = Vz[..., :-1] * (1 - gx) + Vz[..., 1:] * gx
                    l2 += w * float(np.sum((uh - ue[qx::npts]) ** 2))
                    semi += w * float(np.sum((dx - uxe[qx::npts]) ** 2 + dy ** 2 + dz ** 2))
    return float(np.sqrt(l2)), float(np.sqrt(l2 + semi))


def bench_ex52(args, torch, eife):
    """Example 5.2 (Section 5.1), the traveling wave of Table 4: u_t = Lap u + (u - u^3)/eps^2 on
    (0, sqrt 2) x (0, 1/8)^2, eps = 0.05, nonhomogeneous Dirichlet data from the exact wave, entering
    as part of f, T = 3 sqrt(2) eps / 5.  FP64.  Spatial rows: EIFE2, N_T = 1024 on 64x4x4 ... 512x32x32;
    temporal rows: EIFE1 and EIFE2, N_T = 16 ... 128 on 1024x64x64.  Per run: continuous L2 and H1 errors
    (4^3 Gauss points per element) and DoF-steps/s; rates between consecutive rows."""
    eps = 0.05
    T = 3.0 * np.sqrt(2.0) * eps / 5.0
    w2 = 2.0 * np.sqrt(2.0) * eps

    def run(nx, ny, nt, stages):
        N = [nx, ny, ny]
        h = [np.sqrt(2.0) / nx, 0.125 / ny, 0.125 / ny]
        x = h[0] * np.arange(1, nx)
        u0 = np.broadcast_to(0.5 * (1.0 - np.tanh(x / w2)), (ny - 1, ny - 1, nx - 1))
        g = eife.Grid(N, h, 1.0, "f64")
        g.set_forcing(eps, 0.0)
        g.set_phi(T / nt, stages)
        u = torch.tensor(np.ascontiguousarray(u0), device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(u, nt, eife.F_TRAVELING_WAVE, 0.0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        g.close()
        l2, h1 = q1_errors_wave(u.cpu().numpy(), N, h, T, eps)
        ndof = (nx - 1) * (ny - 1) ** 2
        log(f"  EIFE{stages} N_T={nt} {nx}x{ny}x{ny}: L2 {l2:.4e} H1 {h1:.4e}, {ndof * nt / dt:.3e} DoF-steps/s")
        return {"N_T": nt, "grid": f"{nx}x{ny}x{ny}", "L2": l2, "H1": h1, "dof_steps_per_s": ndof * nt / dt}

    def with_rates(rows):
        for a, b in zip(rows, rows[1:]):
            b["L2_rate"] = round(float(np.log2(a["L2"] / b["L2"])), 2)
            b["H1_rate"] = round(float(np.log2(a["H1"] / b["H1"])), 2)
        return rows

    log("bench: Example 5.2 traveling wave (Table 4), FP64")
    res = {"spatial_eife2": with_rates([run(nx, nx // 16, 1024, 2) for nx in (64, 128, 256, 512)])}
    for stages in (1, 2):
        res[f"temporal_eife{stages}"] = with_rates([run(1024, 64, nt, stages) for nt in (16, 32, 64, 128)])
    for key, rows in res.items():
        for r in rows:
            log(f"  {key:15s} N_T={r['N_T']:5d} {r['grid']:>11s} L2 {r['L2']:.4e} ({r.get('L2_rate', '-')}) "
                f"H1 {r['H1']:.4e} ({r.get('H1_rate', '-')}) {r['dof_steps_per_s']:.3e} DoF-steps/s")
    best = res["temporal_eife2"][-1]
    ndof = 1023 * 63 * 63
    cpu = None
    if not args.no_cpu:
        from oracle import problems, spectral, stepper
        cores = cpu_cores()
        nx, ny = 512, 32
        Ns, hs = [nx, ny, ny], [np.sqrt(2.0) / nx, 0.125 / ny, 0.125 / ny]
        basis = spectral.SineBasis(Ns, hs, 1.0, workers=cores)
        uw, uwt, _ = problems.traveling_wave_solution(eps)
        x = hs[0] * np.arange(1, nx)
        u0s = np.broadcast_to(uw(0.0, x), (ny - 1, ny - 1, nx - 1))
        bd = (lambda t, Xb: uw(t, Xb[0]), lambda t, Xb: uwt(t, Xb[0]))
        tau = T / 1024
        cpu = cpu_oracle_rate(
            lambda: stepper.run(basis, u0s, problems.traveling_wave(eps), tau, 1, 2, boundary=bd),
            lambda U, k: stepper.run(basis, U, problems.traveling_wave(eps), tau, k, 2, t0=tau, boundary=bd),
            (nx - 1) * (ny - 1) ** 2, 15.0, 200, cores,
            "{steps} EIFE2 steps of Table 4's 512x32x32 spatial row (N_T = 1024; after 1 untimed step; the "
            "1024x64x64 grid's all-node boundary matrices are too large for the oracle; each oracle call builds "
            "the boundary matrices once, inside the timing), FP64 oracle tier C "
            f"(scipy.fft.dstn, workers={cores}), {{dt:.2f}} s")
        log(f"bench: cpu oracle {cpu['value']:.4e} DoF-steps/s on {cpu['cores']} cores")
    out = {"metric": "Example 5.2 (Table 4) EIFE errors, observed rates and DoF-steps/s", "value": best["dof_steps_per_s"],
           "unit": "DoF-steps/s", "n_gpus": 1, "steps": best["N_T"], "warmup": 0,
           "ms_per_step": 1e3 * ndof / best["dof_steps_per_s"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "Example 5.2 traveling wave, eps=0.05, nonhomogeneous Dirichlet data as part of f, "
                                  "T=3 sqrt(2) eps/5; value: EIFE2 N_T=128 on 1024x64x64", "dofs": ndof},
           "ex52": res, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    return 0


def bench_variable(args, torch, eife):
    """Variable step sizes on the benchmark problem (3D Allen-Cahn 255^3 FP32 EIFE2): the same
    K steps through eife_step (uniform tau) and through eife_step_variable with equal steps
    (same bits) and with varying steps tau_n = tau (1 + 0.5 sin n); DoF-steps/s of each, so the
    cost of the per-step factors (built on the host, staged in chunks) shows."""
    N = [N_INT] * 3
    h = [1.0 / N_INT] * 3
    ndof = (N_INT - 1) ** 3
    u0 = seeded_inputs.uniform_field(SEED, N)
    K = args.steps
    g = eife.Grid(N, h, EPS * EPS, "f32")
    g.set_phi(TAU, 2)
    u = torch.tensor(u0, dtype=torch.float32, device="cuda")
    g.step(u, args.warmup, eife.F_ALLEN_CAHN, 0.0)
    g.step_variable(u, [TAU] * max(args.warmup, 1), eife.F_ALLEN_CAHN, 0.0)
    res = {}
    runs = (("uniform_eife_step", None), ("equal_taus_step_variable", [TAU] * K),
            ("varying_taus_step_variable", list(TAU * (1.0 + 0.5 * np.sin(np.arange(K))))))
    outs = {}
    for name, taus in runs:
        u.copy_(torch.tensor(u0, dtype=torch.float32))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if taus is None:
            g.step(u, K, eife.F_ALLEN_CAHN, 0.0)
        else:
            g.step_variable(u, taus, eife.F_ALLEN_CAHN, 0.0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        outs[name] = u.clone()
        res[name] = {"dof_steps_per_s": ndof * K / dt, "ms_per_step": dt * 1e3 / K}
        log(f"  {name:28s} {dt * 1e3 / K:.4f} ms/step, {ndof * K / dt:.4e} DoF-steps/s")
    g.close()
    res["equal_taus_bitwise_equal"] = bool(torch.equal(outs["uniform_eife_step"], outs["equal_taus_step_variable"]))
    v = res["varying_taus_step_variable"]
    cpu = None
    if not args.no_cpu:
        from oracle import problems, spectral, stepper
        cores = cpu_cores()
        basis = spectral.SineBasis(N, h, EPS * EPS, workers=cores)
        taus = list(TAU * (1.0 + 0.5 * np.sin(np.arange(K))))
        cpu = cpu_oracle_rate(
            lambda: stepper.run(basis, u0, problems.allen_cahn(), taus[:1], 1, 2),
            lambda U, k: stepper.run(basis, U, problems.allen_cahn(), taus[1:1 + k], k, 2, t0=taus[0]), ndof, 15.0,
            min(20, K - 1), cores,
            "{steps} varying-step EIFE2 steps of the same 255^3 problem (after 1 untimed step), FP64 oracle tier C "
            f"(scipy.fft.dstn, workers={cores}), {{dt:.2f}} s")
        log(f"bench: cpu oracle {cpu['value']:.4e} DoF-steps/s on {cpu['cores']} cores")
    out = {"metric": "variable-step EIFE2 DoF-steps/s", "value": v["dof_steps_per_s"], "unit": "DoF-steps/s",
           "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": v["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "3D Allen-Cahn eps=0.02, 255^3 DoFs, FP32, EIFE2 c2=1/2, tau_n = 0.005 (1 + 0.5 sin n)",
                      "dofs": ndof},
           "variable": res, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    return 0


def bench_three(args, torch, eife):
    """The three-stage scheme (eq. (2.2), nodes 0, 1/3, 2/3): (1) throughput on the benchmark problem
    (3D Allen-Cahn 255^3 FP32) next to EIFE2 with per-pass event timings; (2) temporal errors on the
    manufactured problem (2D 1023^2 FP64, T = 1) against a same-grid three-stage run at tau = 2^-10,
    for EIFE2 and the three-stage scheme, with the observed orders."""
    N = [N_INT] * 3
    h = [1.0 / N_INT] * 3
    ndof = (N_INT - 1) ** 3
    u0 = seeded_inputs.uniform_field(SEED, N)
    K = args.steps
    res = {"cube": {}}
    # FP32 bytes per DoF per launch: the first three-stage pass reads W, H and writes W, H, X; the
    # second reads W, H, X and writes W, H; the third reads and writes W, H
    s3_bytes = {"last_a": 20, "last_b": 18}
    for stages in (2, 3):
        g = eife.Grid(N, h, EPS * EPS, "f32")
        g.set_phi(TAU, stages)
        u = torch.tensor(u0, dtype=torch.float32, device="cuda")
        g.step(u, args.warmup, eife.F_ALLEN_CAHN, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(u, K, eife.F_ALLEN_CAHN, 0.0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        g.profile(True)
        g.step(u, min(K, 20), eife.F_ALLEN_CAHN, 0.0)
        prof = g.profile_read()
        g.profile(False)
        g.close()
        passes = {}
        for name, (ms, cnt) in prof.items():
            if cnt:
                b = s3_bytes.get(name, BYTES_PER_DOF[name]) if stages == 3 else BYTES_PER_DOF[name]
                passes[name] = {"launches": cnt, "avg_us": round(ms / cnt * 1e3, 2),
                                "alg_GBs": round(b * ndof / (ms / cnt * 1e-3) / 1e9, 1)}
        res["cube"][f"stages{stages}"] = {"ms_per_step": dt * 1e3 / K, "dof_steps_per_s": ndof * K / dt,
                                          "passes": passes}
        log(f"  {stages} stages, 255^3 FP32: {dt * 1e3 / K:.3f} ms/step, {ndof * K / dt:.4e} DoF-steps/s; "
            + ", ".join(f"{k} {v['avg_us']} us ({v['alg_GBs']} GB/s)" for k, v in passes.items()))
        del u
    # temporal orders on the manufactured problem
    n_int = 1024
    Nm, hm = [n_int, n_int], [1.0 / n_int] * 2
    sx = np.sin(np.pi * np.arange(1, n_int) / n_int)
    base = np.outer(sx, sx)

    def run(stages, k):
        g = eife.Grid(Nm, hm, 1.0, "f64")
        g.set_phi(2.0 ** -k, stages)
        u = torch.tensor(base, device="cuda")
        g.step(u, 2 ** k, eife.F_MMS_U2, 0.0)
        torch.cuda.synchronize()
        return g, u

    g_ref, u_ref = run(3, 10)
    rows = {}
    for stages in (2, 3):
        errs = []
        for k in (3, 4, 5, 6):
            g, u = run(stages, k)
            errs.append(g.norms(u, u_ref)[0])
            g.close()
        rates = [round(float(np.log2(a / b)), 2) for a, b in zip(errs, errs[1:])]
        rows[f"stages{stages}"] = {"tau": [2.0 ** -k for k in (3, 4, 5, 6)], "L2_vs_ref": errs, "rates": rates}
        log(f"  manufactured 1023^2 FP64, {stages} stages: L2 vs tau=2^-10 three-stage run "
            + " ".join(f"{e:.3e}" for e in errs) + f", rates {rates}")
    g_ref.close()
    res["manufactured_orders"] = rows
    cpu = None
    if not args.no_cpu:
        from oracle import erk, problems, spectral
        cores = cpu_cores()
        basis = spectral.SineBasis(N, h, EPS * EPS, workers=cores)
        nodes = [0.0, 1.0 / 3.0, 2.0 / 3.0]
        cpu = cpu_oracle_rate(
            lambda: erk.run(basis, u0, problems.allen_cahn(), TAU, 1, nodes),
            lambda U, k: erk.run(basis, U, problems.allen_cahn(), TAU, k, nodes, t0=TAU), ndof, 15.0, 10, cores,
            "{steps} three-stage steps of the same 255^3 problem (after 1 untimed step), FP64 oracle (oracle/erk.py, "
            f"tier C scipy.fft.dstn, workers={cores}), {{dt:.2f}} s")
        log(f"bench: cpu oracle {cpu['value']:.4e} DoF-steps/s on {cpu['cores']} cores")
    v = res["cube"]["stages3"]
    out = {"metric": "three-stage EIFE DoF-steps/s and observed temporal order", "value": v["dof_steps_per_s"],
           "unit": "DoF-steps/s", "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": v["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "3D Allen-Cahn eps=0.02, 255^3 DoFs, FP32, three stages (nodes 0, 1/3, 2/3), "
                                  "tau=0.005", "dofs": ndof},
           "three_stage": res, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    return 0


# Table 3 of the paper (Example 5.1, EIFE2 with c2 = 1/2, N_T = 50): average seconds per step of the
# authors' Matlab FP64 solver on an Intel i5-8250U (1.8 GHz, 8 GB), per grid of intervals.
PAPER_TABLE3 = {(512, 256): 1.121, (1024, 512): 4.444, (2048, 1024): 17.516, (4096, 2048): 75.944}


def bench_longlines(args, torch, eife):
    """The long-line passes on the manufactured problem's grid: 4096^2 intervals (4095^2 DoFs,
    8192-point odd extensions on both axes), EIFE2 tau = 2^-10 from the exact initial state,
    FP32 and FP64.  Per precision: K timed steps in one call after a settle and warm-up, then a
    second run of K steps with per-pass event timing and each pass's algorithmic HBM rate
    (x pass: W read and written; y stage passes: W and H read and written)."""
    n_int = 4096
    N, h = [n_int, n_int], [1.0 / n_int] * 2
    ndof = (n_int - 1) ** 2
    tau = 2.0 ** -10
    steps = args.steps if args.steps != 200 else 20
    warm = args.warmup if args.warmup != 20 else 5
    s1 = np.sin(np.pi * np.arange(1, n_int) / n_int)
    base = np.outer(s1, s1)
    out = {}
    log(f"bench: long lines, manufactured 2D {n_int - 1}^2 DoFs, EIFE2 tau=2^-10, steps={steps}")
    for dt, tdt, esz in (("f32", torch.float32, 4), ("f64", torch.float64, 8)):
        g = eife.Grid(N, h, 1.0, dt)
        g.set_phi(tau, 2)
        u = torch.tensor(base, dtype=tdt, device="cuda")
        if args.settle > 0:
            settle(torch, g, u, eife.F_MMS_U2, min(args.settle, 0.5), chunk=10)
        g.step(u, warm, eife.F_MMS_U2, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(u, steps, eife.F_MMS_U2, warm * tau)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        g.profile(True)
        g.step(u, steps, eife.F_MMS_U2, (warm + steps) * tau)
        prof = g.profile_read()
        g.profile(False)
        torch.cuda.synchronize()
        g.close()
        passes = {}
        for name, (ms, cnt) in prof.items():
            if cnt == 0:
                continue
            avg = ms / cnt * 1e-3
            nbytes = BYTES_PER_DOF[name] * (esz // 4) * ndof
            gbs = nbytes / avg / 1e9
            passes[name] = {"launches": cnt, "avg_us": round(avg * 1e6, 2), "bytes_per_launch": nbytes,
                            "alg_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
            log(f"  {dt} pass {name:10s} launches={cnt:5d} avg={avg * 1e6:8.2f} us alg={gbs:8.1f} GB/s "
                f"({gbs / HBM_PEAK_GBS * 100:5.1f}% of HBM peak)")
        out[dt] = {"ms_per_step": round(wall * 1e3, 4), "dof_steps_per_s": ndof / wall, "passes": passes}
        log(f"bench: {dt} {wall * 1e3:.3f} ms/step, {ndof / wall:.4e} DoF-steps/s")
    dom = max(out["f32"]["passes"].items(), key=lambda kv: kv[1]["avg_us"] * kv[1]["launches"])
    line = {"metric": "long-line EIFE2 DoF-steps/s (4095^2 manufactured problem, 8192-point lines)",
            "value": out["f32"]["dof_steps_per_s"], "unit": "DoF-steps/s", "n_gpus": 1, "steps": steps,
            "warmup": warm, "ms_per_step": out["f32"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "manufactured 2D u_t = Lap u + u^2 + g, 4096^2 intervals, EIFE2 tau = 2^-10, "
                                   "exact initial state; value: FP32 (FP64 under 'f64')", "dofs": ndof},
            "roofline": {"bound": "hbm", "achieved": dom[1]["alg_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": dom[1]["frac"], "traffic": None, "kernel": dom[0],
                         "kernel_avg_us": dom[1]["avg_us"], "bytes_per_launch": dom[1]["bytes_per_launch"]},
            "cpu_baseline": None, "f32": out["f32"], "f64": out["f64"]}
    print(json.dumps(line), flush=True)


def bench_table3(args, torch, eife):
    """The paper's timing table (Table 3): Example 5.1, u_t = (1/2) Lap u - (pi^2/2) u + (pi^2/2) e^{-pi^2 t}
    sin(pi x) sin(pi y) on (1/2, 5/2) x (0, 1), exact u = e^{-pi^2 t} (sin(pi x) - 1) sin(pi y), EIFE2 with
    c2 = 1/2 and N_T = 50 (tau = 1/50, T = 1), FP64, grids 512x256 ... 4096x2048 intervals.  Per grid: the
    50 steps timed in one call (after one untimed call), DoF-steps/s next to the paper's Matlab figure on
    its laptop CPU, and the discrete L2 error against the exact nodal values at T as a check."""
    rows = []
    log("bench: Table 3 (Example 5.1, EIFE2, N_T = 50, FP64)")
    for (nx, ny), paper_s in PAPER_TABLE3.items():
        N, h = [nx, ny], [2.0 / nx, 1.0 / ny]
        x = 0.5 + h[0] * np.arange(1, nx)
        y = h[1] * np.arange(1, ny)
        base = np.outer(np.sin(np.pi * y), np.sin(np.pi * x) - 1.0)  # [y][x]
        g = eife.Grid(N, h, 0.5, "f64")
        g.set_origin([0.5, 0.0])
        g.set_phi(1.0 / 50.0, 2)
        u = torch.tensor(base, device="cuda")
        g.step(u, 50, eife.F_EX51, 0.0)  # untimed
        u.copy_(torch.tensor(base))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(u, 50, eife.F_EX51, 0.0)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 50
        exact = torch.tensor(np.exp(-np.pi ** 2) * base, device="cuda")
        l2 = g.norms(u, exact)[0]
        g.close()
        ndof = (nx - 1) * (ny - 1)
        row = {"grid": f"{nx}x{ny}", "dofs": ndof, "s_per_step": dt, "dof_steps_per_s": ndof / dt,
               "paper_s_per_step": paper_s, "paper_dof_steps_per_s": ndof / paper_s, "speedup_vs_paper": paper_s / dt,
               "L2_vs_exact_nodal": l2}
        rows.append(row)
        log(f"  {nx}x{ny}: {dt * 1e3:.4f} ms/step, {ndof / dt:.4e} DoF-steps/s; paper {paper_s:.3f} s/step "
            f"({ndof / paper_s:.3e} DoF-steps/s, i5-8250U Matlab) -> x{paper_s / dt:.0f}; L2 vs exact {l2:.3e}")
    cpu = None
    if not args.no_cpu:
        from oracle import problems, spectral, stepper
        cores = cpu_cores()
        nx, ny = 2048, 1024
        N, h = [nx, ny], [2.0 / nx, 1.0 / ny]
        x = 0.5 + h[0] * np.arange(1, nx)
        y = h[1] * np.arange(1, ny)
        base = np.outer(np.sin(np.pi * y), np.sin(np.pi * x) - 1.0)
        basis = spectral.SineBasis(N, h, 0.5, workers=cores)
        cpu = cpu_oracle_rate(
            lambda: stepper.run(basis, base, problems.ex51(), 1.0 / 50, 1, 2, origin=(0.5, 0.0)),
            lambda U, k: stepper.run(basis, U, problems.ex51(), 1.0 / 50, k, 2, t0=1.0 / 50, origin=(0.5, 0.0)),
            (nx - 1) * (ny - 1), 12.0, 49, cores,
            "{steps} EIFE2 steps of Table 3's 2048x1024 grid (after 1 untimed step), FP64 oracle tier C "
            f"(scipy.fft.dstn, workers={cores}), {{dt:.2f}} s")
        log(f"bench: cpu oracle {cpu['value']:.4e} DoF-steps/s on {cpu['cores']} cores")
    big = rows[-1]
    out = {"metric": "Table 3 (Example 5.1) EIFE2 DoF-steps/s per grid, with the paper's Matlab timings",
           "value": big["dof_steps_per_s"], "unit": "DoF-steps/s", "n_gpus": 1, "steps": 50, "warmup": 50,
           "ms_per_step": big["s_per_step"] * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": big["speedup_vs_paper"], "dtype": "f64", "data": "synthetic",
           "config": {"workload": "Example 5.1 (Table 3), EIFE2 c2=1/2, N_T=50, FP64; value: 4096x2048 intervals; "
                                  "vs_baseline: against the paper's 75.944 s/step (Matlab FP64, Intel i5-8250U "
                                  "1.8 GHz laptop)", "dofs": big["dofs"]},
           "table3": rows, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--workload", choices=["cube", "batched", "manufactured", "ex53", "ex52", "variable", "three", "table3",
                                           "corrnet", "longlines"], default="cube",
                    help="cube: 3D Allen-Cahn 255^3 (default line); batched: 512 independent 2D instances; "
                         "manufactured: 4095^2 orders, errors and rates; ex53: periodic 128^3 Flory-Huggins "
                         "grain coarsening to T = 20; ex52: traveling wave with Dirichlet data (Table 4); "
                         "variable: the cube problem with varying step sizes; three: the three-stage scheme; "
                         "table3: the paper's timing table (Example 5.1); corrnet: the corrector network's "
                         "kernels alone (matrix-core rate); longlines: the 4095^2 manufactured grid's "
                         "8192-point line passes, per-pass HBM rates")
    ap.add_argument("--transform", choices=["fft", "gemm"], default="fft",
                    help="cube workload: FFT sine transforms (default) or split-BF16 matrix-core products")
    ap.add_argument("--no-corrector", action="store_true",
                    help="skip the learned-corrector comparison (2D Allen-Cahn 511^2, plain vs corrected EIFE2)")
    ap.add_argument("--corr-seeds", type=int, default=10, help="unseen seeds of the corrector comparison (a plain step must meet the bound on all of them)")
    ap.add_argument("--settle", type=float, default=SETTLE_S,
                    help="seconds of untimed stepping before the warm-up (0 for counter runs, which record "
                         "every dispatch)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run a plain device copy of one work array's size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the EIFE path here is built and timed on a single MI355X "
              "(multi-GPU sharding is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2209_11922_amd as eife

    if args.workload == "batched":
        return bench_batched(args, torch, eife)
    if args.workload == "manufactured":
        return bench_manufactured(args, torch, eife)
    if args.workload == "ex53":
        return bench_ex53(args, torch, eife)
    if args.workload == "ex52":
        return bench_ex52(args, torch, eife)
    if args.workload == "variable":
        return bench_variable(args, torch, eife)
    if args.workload == "three":
        return bench_three(args, torch, eife)
    if args.workload == "table3":
        return bench_table3(args, torch, eife)
    if args.workload == "corrnet":
        return bench_corrnet(args, torch, eife)
    if args.workload == "longlines":
        return bench_longlines(args, torch, eife)

    N = [N_INT] * 3
    h = [1.0 / N_INT] * 3
    D = EPS * EPS
    ndof = (N_INT - 1) ** 3
    u0 = seeded_inputs.uniform_field(SEED, N)
    log(f"bench: 3D Allen-Cahn {N_INT - 1}^3 FP32 EIFE2 tau={TAU} warmup={args.warmup} steps={args.steps}")

    if args.copy_calib:
        # one elementwise kernel that reads and writes ndof floats once each
        a = torch.ones(ndof, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        log(f"bench: calibration copy (torch.mul) reading and writing {ndof * 4} bytes, x3")
        del a, b
    g = eife.Grid(N, h, D, "f32")
    gemm = args.transform == "gemm"
    if gemm:
        g.set_transform(eife.binding.TX_GEMM_SPLITBF16)
    g.set_phi(TAU, 2)
    u = torch.tensor(u0, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    settled = settle(torch, g, u, eife.F_ALLEN_CAHN, args.settle) if args.settle > 0 else 0
    log(f"bench: settle {settled} untimed steps on a scratch copy ({args.settle:.1f} s)")
    if args.warmup > 0:
        g.step(u, args.warmup, eife.F_ALLEN_CAHN, 0.0)
    torch.cuda.synchronize()
    t_start = args.warmup * TAU
    t0 = time.perf_counter()
    g.step(u, args.steps, eife.F_ALLEN_CAHN, t_start)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = ndof * args.steps / dt
    log(f"bench: {dt * 1e3 / args.steps:.3f} ms/step, {value:.4e} DoF-steps/s")

    # achievable streaming bandwidth: a plain device copy of one work array's
    # size (read + write), event-timed after the measured run
    a = torch.ones(ndof, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    copy_gbs = 2 * ndof * 4 * 20 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    log(f"bench: plain device copy {copy_gbs:.1f} GB/s ({copy_gbs / HBM_PEAK_GBS * 100:.1f}% of HBM peak)")

    # per-pass event timing over a second run of the same K steps
    if args.settle > 0:
        settle(torch, g, u, eife.F_ALLEN_CAHN, min(args.settle, 0.3))
    g.profile(True)
    g.step(u, args.steps, eife.F_ALLEN_CAHN, t_start + args.steps * TAU)
    prof = g.profile_read()
    g.profile(False)
    torch.cuda.synchronize()
    rows = []
    for name, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        avg_ms = ms / cnt
        gbs = BYTES_PER_DOF[name] * ndof / (avg_ms * 1e-3) / 1e9
        rows.append((ms, name, cnt, avg_ms, gbs))
        log(f"  pass {name:10s} launches={cnt:5d} total={ms:9.3f} ms avg={avg_ms * 1e3:8.2f} us "
            f"alg={gbs:8.1f} GB/s ({gbs / HBM_PEAK_GBS * 100:5.1f}% of HBM peak)")
    rows.sort(reverse=True)
    dom = rows[0]
    prof_step_ms = sum(r[0] for r in rows) / args.steps
    step_bytes = sum(BYTES_PER_DOF[r[1]] * r[2] for r in rows) * ndof / args.steps
    log(f"  profiled step {prof_step_ms:.3f} ms; whole-step algorithmic bandwidth "
        f"{step_bytes / (dt / args.steps) / 1e9:.1f} GB/s")
    roof = {"bound": "hbm", "achieved": round(dom[4], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(dom[4] / HBM_PEAK_GBS, 4), "traffic": None if gemm else measured_traffic(dom[1]),
            "kernel": dom[1], "kernel_avg_us": round(dom[3] * 1e3, 2),
            "bytes_per_launch": BYTES_PER_DOF[dom[1]] * ndof,
            "step_achieved_GBs": round(step_bytes / (dt / args.steps) / 1e9, 1),
            "copy_GBs": round(copy_gbs, 1), "frac_of_copy": round(dom[4] / copy_gbs, 4)}
    if gemm:
        # matrix-core view: 3 BF16 products of 2 (N-1) flops per DoF per transform
        gemms = GEMMS_PER_PASS[dom[1]]
        flops = gemms * 3 * 2 * (N_INT - 1) * ndof
        tfs = flops / (dom[3] * 1e-3) / 1e12
        roof["mfma"] = {"achieved": round(tfs, 1), "peak": BF16_PEAK_TFS, "unit": "TFLOP/s",
                        "frac": round(tfs / BF16_PEAK_TFS, 4), "flops_per_launch": flops}
        log(f"  dominant pass {dom[1]}: {tfs:.1f} TFLOP/s BF16 ({tfs / BF16_PEAK_TFS * 100:.1f}% of dense peak)")

    red = reduction_rate(torch, g, u, ndof)
    g.close()
    del u
    acc = accuracy_vs_f64(torch, eife, u0, N, h, D, args.steps)
    f64 = None if gemm else f64_rate(torch, eife, u0, N, h, D, args.steps, args.settle)

    corr = None
    if not args.no_corrector and not gemm:
        corr = corrector_comparison(args.corr_seeds)

    cpu = None
    if not args.no_cpu and not gemm:
        cpu = cpu_baseline(u0, N, h, D)
        log(f"bench: cpu oracle {cpu['value']:.4e} DoF-steps/s on {cpu['cores']} cores")

    out = {"metric": METRIC, "value": value, "unit": "DoF-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "settle_steps": settled, "ms_per_step": dt * 1e3 / args.steps,
           "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3+f32acc" if gemm else "f32", "data": "synthetic",
           "config": {"workload": "3D Allen-Cahn eps=0.02, Q1 grid 256^3 intervals (255^3 DoFs), Dirichlet, "
                                  "u0 uniform[-0.9,0.9] seed 0, EIFE2 c2=1/2 tau=0.005, "
                                  + ("split-BF16 matrix-core sine transforms" if gemm else "FP32 sine-transform path"),
                      "dofs": ndof, "tau": TAU, "scheme": "EIFE2", "transform": args.transform},
           "roofline": roof, "cpu_baseline": cpu, "accuracy": acc, "corrector": corr, "reductions": red,
           "f64": f64,
           # the paper's only timings (Table 3), another workload on other hardware: context only
           "paper_timings": {"table": "Table 3, Example 5.1 (2D), EIFE2, N_T = 50, FP64",
                             "hardware": "Matlab on an Intel i5-8250U 1.8 GHz laptop, 8 GB",
                             "s_per_step": {f"{nx}x{ny}": t for (nx, ny), t in PAPER_TABLE3.items()},
                             "dof_steps_per_s": {f"{nx}x{ny}": round((nx - 1) * (ny - 1) / t, 1)
                                                 for (nx, ny), t in PAPER_TABLE3.items()},
                             "same_workload_here": "bench.py --workload table3"}}
    print(json.dumps(out), flush=True)


CORR_FLOP_PER_NODE = 2 * 9 * (2 * 32 + 4 * 32 * 32 + 32)  # six 3x3 layers, 2 -> 32 -> ... -> 32 -> 1


def bench_corrnet(args, torch, eife):
    """The learned corrector's network alone (2D 511^2, the committed trained weights): the
    BF16 matrix-core forward (inference) and the forward + backward of a training gradient,
    event-timed on the stream the kernels run on; only the network's kernels are launched."""
    from paper_2209_11922_amd import corrector as cor
    n = 511
    steps = args.steps if args.steps != 200 else 50
    warm = args.warmup if args.warmup != 20 else 5
    p, s_out, _, _ = cor.load(os.path.join(ROOT, "paper_2209_11922_amd", "weights", "corrector_ac512.npz"))
    B = 8
    net = eife.Corrector(n, n, B)
    net.set_params(p)
    net.set_scale(s_out)
    un = torch.tensor(np.stack([seeded_inputs.uniform_field(s, [n + 1, n + 1]) for s in range(B)]),
                      dtype=torch.float32, device="cuda")
    uc = (0.99 * un).contiguous()
    uf = (0.985 * un).contiguous()
    stream = torch.cuda.current_stream()
    flop1 = CORR_FLOP_PER_NODE * n * n
    out = {}
    for name, batch in (("forward_b1", 1), ("forward_b8", B)):
        a, b = (un[0], uc[0]) if batch == 1 else (un, uc)
        d = torch.empty_like(b)
        for _ in range(warm):
            net.forward(a, b, d, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            net.forward(a, b, d, stream=stream)
        e1.record(stream)
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / steps
        tfs = flop1 * batch / (us * 1e-6) / 1e12
        out[name] = {"us_per_call": round(us, 2), "TFLOPs": round(tfs, 1), "frac": round(tfs / BF16_PEAK_TFS, 4),
                     "flop_per_call": flop1 * batch}
        log(f"bench: corrector {name}: {us:.1f} us per call, {tfs:.1f} TFLOP/s BF16 "
            f"({tfs / BF16_PEAK_TFS * 100:.1f}% of dense peak)")
    # training gradient (forward + data and weight gradients, about 3x the forward's work) at batch 8
    for _ in range(max(1, warm // 2)):
        net.grad(un, uc, uf, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(1, steps // 5)
    for _ in range(reps):
        net.grad(un, uc, uf, stream=stream)  # returns the gradient to the host (one wait per call)
    dt = (time.perf_counter() - t0) / reps
    tfs = 3 * flop1 * B / dt / 1e12
    out["grad_b8"] = {"us_per_call": round(dt * 1e6, 1), "TFLOPs": round(tfs, 1), "frac": round(tfs / BF16_PEAK_TFS, 4),
                      "flop_per_call": 3 * flop1 * B, "note": "wall time per call, gradient copied to the host"}
    log(f"bench: corrector grad_b8: {dt * 1e6:.1f} us per call, {tfs:.1f} TFLOP/s BF16 (wall)")
    best = out["forward_b8"]
    line = {"metric": "corrector network BF16 TFLOP/s (forward, 2D 511^2)", "value": best["TFLOPs"],
            "unit": "TFLOP/s", "n_gpus": 1, "steps": steps, "warmup": warm, "ms_per_step": best["us_per_call"] / 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f32acc",
            "data": "synthetic",
            "config": {"workload": "learned-corrector network, 6 3x3 conv layers 2-32-32-32-32-32-1, 511^2 nodes, "
                                   "trained weights, batch 8 (and 1)", "flop_per_node": CORR_FLOP_PER_NODE},
            "roofline": {"bound": "mfma", "achieved": best["TFLOPs"], "peak": BF16_PEAK_TFS, "unit": "TFLOP/s",
                         "frac": best["frac"], "traffic": None, "kernel": "whole forward (9 kernels)"},
            "cpu_baseline": None, "calls": out}
    print(json.dumps(line), flush=True)
    net.close()


def bench_batched(args, torch, eife):
    """512 independent 2D Allen-Cahn instances, N ~ U{128,192,256,384,512}, eps ~ U[0.01, 0.05],
    EIFE2 tau = 0.01, FP32 with double phi factors, launch shapes from the autotuner."""
    draws = seeded_inputs.batch_instances(0, 512)
    grids = [(n, n, 1.0 / n, 1.0 / n, e * e) for n, e, _ in draws]
    ndof = sum((n - 1) ** 2 for n, _, _ in draws)
    steps = args.steps if args.steps != 200 else 50
    warm = args.warmup if args.warmup != 20 else 1
    log(f"bench: batched 512 instances, {ndof} DoFs, EIFE2 tau=0.01, FP32, steps={steps}")
    b = eife.Batch(grids, "f32")
    b.set_phi(0.01, 2)
    cache = os.path.join("/tmp", "eife_autotune.json")
    t0 = time.perf_counter()
    b.autotune(cache)
    log(f"bench: autotune {time.perf_counter() - t0:.2f} s, classes (Nx, Ny, count, row var, col var): "
        f"{b.class_info()}")
    u = torch.cat([torch.tensor(seeded_inputs.uniform_field(s, [n, n]).reshape(-1), dtype=torch.float32)
                   for n, _, s in draws]).cuda()
    stream = torch.cuda.current_stream()
    for _ in range(max(1, warm)):
        b.step(u, steps, eife.F_ALLEN_CAHN, 0.0, stream=stream)  # captures, then replays
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(u, steps, eife.F_ALLEN_CAHN, 0.0, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = ndof * steps / dt
    gbs = 48.0 * ndof * steps / dt / 1e9
    log(f"bench: batched {dt * 1e3 / steps:.3f} ms/step, {value:.4e} DoF-steps/s, {gbs:.0f} GB/s algorithmic "
        f"({gbs / HBM_PEAK_GBS * 100:.1f}% of HBM peak)")
    out = {"metric": METRIC, "value": value, "unit": "DoF-steps/s", "n_gpus": 1, "steps": steps, "warmup": warm,
           "ms_per_step": dt * 1e3 / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "512 independent 2D Allen-Cahn instances, N in {128,192,256,384,512}, "
                                  "eps in [0.01,0.05], EIFE2 tau=0.01, one graph replay", "dofs": ndof},
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "whole step (48 B/DoF)"},
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)
    b.close()


if __name__ == "__main__":
    main()
