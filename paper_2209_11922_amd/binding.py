"""ctypes binding of the C ABI declared in include/eife.h (argument marshalling only)."""
import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB = None

# status codes
OK, EINVAL, ENOMEM, EUNSUPPORTED, ESTATE, EHIP, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
# enums
BC_DIRICHLET, BC_PERIODIC = 0, 1
F32, F64 = 0, 1
F_ZERO, F_ALLEN_CAHN, F_MMS_U2, F_EX51, F_CONST, F_AFFINE_T, F_FLORY_HUGGINS, F_TRAVELING_WAVE = range(8)
LOAD_LUMPED, LOAD_NODAL = 0, 1
TX_FFT, TX_FFT_GENERIC, TX_GEMM_SPLITBF16 = 0, 1, 2
PASS_NAMES = ["row_phys", "row_fwd", "row_inv", "mid", "last_plain", "last_a", "last_b", "last_etd1"]

_DTYPES = {"f32": (F32, torch.float32), "f64": (F64, torch.float64),
           torch.float32: (F32, torch.float32), torch.float64: (F64, torch.float64)}


class EIFEError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"eife error {code}: {msg}")
        self.code = code


def library_path():
    return os.path.join(_PKG, "libeife.so")


def load_library():
    """Load libeife.so from the package directory; raise if it is not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2209_11922_amd.build")
    lib = ctypes.CDLL(path)
    c_int, c_double, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    lib.eife_create_grid.argtypes = [c_int, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(c_double), c_double,
                                     c_int, c_int, ctypes.POINTER(c_void_p)]
    lib.eife_destroy_grid.argtypes = [c_void_p]
    lib.eife_set_phi.argtypes = [c_void_p, c_double, c_int]
    lib.eife_set_c2.argtypes = [c_void_p, c_double]
    lib.eife_set_origin.argtypes = [c_void_p, ctypes.POINTER(c_double)]
    lib.eife_set_load.argtypes = [c_void_p, c_int]
    lib.eife_set_forcing.argtypes = [c_void_p, c_double, c_double]
    lib.eife_set_transform.argtypes = [c_void_p, c_int]
    lib.eife_step.argtypes = [c_void_p, c_void_p, ctypes.c_int64, c_int, c_double, c_void_p]
    lib.eife_step_out.argtypes = [c_void_p, c_void_p, c_void_p, ctypes.c_int64, c_int, c_double, c_void_p]
    lib.eife_norms.argtypes = [c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_double), c_void_p]
    lib.eife_norms_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.eife_set_nodes3.argtypes = [c_void_p, c_double, c_double]
    lib.eife_step_variable.argtypes = [c_void_p, c_void_p, ctypes.POINTER(c_double), ctypes.c_int64, c_int,
                                       c_double, c_void_p]
    lib.eife_energy.argtypes = [c_void_p, c_void_p, c_int, ctypes.POINTER(c_double), c_void_p]
    lib.eife_grid_size.argtypes = [c_void_p, ctypes.POINTER(ctypes.c_int64)]
    lib.eife_profile.argtypes = [c_void_p, c_int]
    lib.eife_profile_read.argtypes = [c_void_p, ctypes.POINTER(c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.eife_create_batch.argtypes = [c_int, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(c_double),
                                      ctypes.POINTER(c_double), c_int, ctypes.POINTER(c_void_p)]
    lib.eife_destroy_batch.argtypes = [c_void_p]
    lib.eife_batch_offsets.argtypes = [c_void_p, ctypes.POINTER(ctypes.c_int64)]
    lib.eife_batch_set_phi.argtypes = [c_void_p, c_double, c_int]
    lib.eife_batch_step.argtypes = [c_void_p, c_void_p, ctypes.c_int64, c_int, c_double, c_void_p]
    lib.eife_batch_autotune.argtypes = [c_void_p, ctypes.c_char_p, c_void_p]
    lib.eife_batch_class_info.argtypes = [c_void_p, c_int, ctypes.POINTER(ctypes.c_int32)]
    f32p = ctypes.POINTER(ctypes.c_float)
    lib.eife_corr_create.argtypes = [c_int, c_int, c_int, ctypes.POINTER(c_void_p)]
    lib.eife_corr_destroy.argtypes = [c_void_p]
    lib.eife_corr_set_params.argtypes = [c_void_p, f32p, ctypes.c_int64]
    lib.eife_corr_get_params.argtypes = [c_void_p, f32p, ctypes.c_int64]
    lib.eife_corr_set_scale.argtypes = [c_void_p, c_double]
    lib.eife_corr_set_guard.argtypes = [c_void_p, c_double]
    lib.eife_corr_set_fused.argtypes = [c_void_p, c_int]
    lib.eife_corr_forward.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]
    lib.eife_corr_grad.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int, f32p, ctypes.POINTER(c_double),
                                   c_void_p]
    lib.eife_corr_train_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_double,
                                         ctypes.POINTER(c_double), c_void_p]
    lib.eife_corr_infer_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_double, ctypes.c_int64, c_double,
                                         ctypes.POINTER(c_int), ctypes.POINTER(c_double), c_void_p]
    lib.eife_corr_run.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double, ctypes.c_int64,
                                  ctypes.c_int64, c_double, ctypes.POINTER(ctypes.c_int64), c_void_p]
    lib.eife_corr_last_error.restype = ctypes.c_char_p
    lib.eife_corr_last_error.argtypes = []
    for name in ("eife_corr_create", "eife_corr_destroy", "eife_corr_set_params", "eife_corr_get_params",
                 "eife_corr_set_scale", "eife_corr_set_guard", "eife_corr_set_fused", "eife_corr_forward",
                 "eife_corr_grad", "eife_corr_train_step", "eife_corr_infer_step", "eife_corr_run"):
        getattr(lib, name).restype = c_int
    lib.eife_last_error.restype = ctypes.c_char_p
    lib.eife_last_error.argtypes = []
    lib.eife_version.argtypes = []
    for name in ("eife_create_grid", "eife_destroy_grid", "eife_set_phi", "eife_set_c2", "eife_set_origin",
                 "eife_set_load", "eife_set_forcing", "eife_step", "eife_step_out", "eife_step_variable", "eife_set_nodes3", "eife_norms", "eife_energy", "eife_grid_size",
                 "eife_version", "eife_profile", "eife_profile_read", "eife_set_transform", "eife_create_batch",
                 "eife_destroy_batch", "eife_batch_offsets", "eife_batch_set_phi", "eife_batch_step",
                 "eife_batch_autotune", "eife_batch_class_info"):
        getattr(lib, name).restype = c_int
    _LIB = lib
    return lib


def _check(lib, code):
    if code != OK:
        raise EIFEError(code, lib.eife_last_error().decode(errors="replace"))


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Grid:
    """A Q1 grid on prod_a [a_a, a_a + N_a h_a] with homogeneous Dirichlet data.

    Mirrors eife_create_grid / eife_set_phi / eife_step / eife_norms; nodal
    arrays are torch tensors on the GPU with shape (N_{d-1}-1, ..., N_0-1).
    """

    def __init__(self, N, h, D, dtype="f64", bc=BC_DIRICHLET):
        self._lib = load_library()
        self.d = len(N)
        self.N = [int(n) for n in N]
        self.h = [float(x) for x in h]
        self.D = float(D)
        self.dtype_code, self.torch_dtype = _DTYPES[dtype]
        self.shape = tuple(n - 1 for n in reversed(self.N))
        Na = (ctypes.c_int32 * self.d)(*self.N)
        ha = (ctypes.c_double * self.d)(*self.h)
        handle = ctypes.c_void_p()
        _check(self._lib, self._lib.eife_create_grid(self.d, Na, ha, self.D, int(bc), self.dtype_code,
                                                     ctypes.byref(handle)))
        self._g = handle

    def close(self):
        if getattr(self, "_g", None):
            self._lib.eife_destroy_grid(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def size(self):
        n = ctypes.c_int64()
        _check(self._lib, self._lib.eife_grid_size(self._g, ctypes.byref(n)))
        return n.value

    def set_phi(self, tau, stages):
        _check(self._lib, self._lib.eife_set_phi(self._g, float(tau), int(stages)))

    def set_c2(self, c2):
        _check(self._lib, self._lib.eife_set_c2(self._g, float(c2)))

    def set_nodes3(self, c2, c3):
        """Nodes (0, c2, c3) of the three-stage scheme (eife_set_nodes3)."""
        _check(self._lib, self._lib.eife_set_nodes3(self._g, float(c2), float(c3)))

    def set_origin(self, a):
        arr = (ctypes.c_double * self.d)(*[float(x) for x in a])
        _check(self._lib, self._lib.eife_set_origin(self._g, arr))

    def set_load(self, kind):
        _check(self._lib, self._lib.eife_set_load(self._g, int(kind)))

    def set_transform(self, kind):
        _check(self._lib, self._lib.eife_set_transform(self._g, int(kind)))

    def set_forcing(self, c0, c1=0.0):
        _check(self._lib, self._lib.eife_set_forcing(self._g, float(c0), float(c1)))

    def _check_array(self, u, name):
        if not isinstance(u, torch.Tensor) or not u.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
        if u.dtype != self.torch_dtype:
            raise TypeError(f"{name} has dtype {u.dtype}, grid expects {self.torch_dtype}")
        if not u.is_contiguous() or u.numel() != self.size():
            raise ValueError(f"{name} must be contiguous with {self.size()} elements")

    def step(self, u, n_steps, f_kind, t0=0.0, stream=None):
        """Advance u in place by n_steps steps (asynchronous on `stream`)."""
        self._check_array(u, "u")
        _check(self._lib, self._lib.eife_step(self._g, ctypes.c_void_p(u.data_ptr()), int(n_steps), int(f_kind),
                                              float(t0), _stream_ptr(stream)))
        return u

    def step_out(self, u_in, u_out, n_steps, f_kind, t0=0.0, stream=None):
        """n_steps steps from u_in into u_out (eife_step_out; u_in is left as it was)."""
        self._check_array(u_in, "u_in")
        self._check_array(u_out, "u_out")
        _check(self._lib, self._lib.eife_step_out(self._g, ctypes.c_void_p(u_in.data_ptr()),
                                                  ctypes.c_void_p(u_out.data_ptr()), int(n_steps), int(f_kind),
                                                  float(t0), _stream_ptr(stream)))
        return u_out

    def step_variable(self, u, taus, f_kind, t0=0.0, stream=None):
        """Advance u in place by len(taus) steps of sizes taus[n] (eife_step_variable)."""
        self._check_array(u, "u")
        arr = (ctypes.c_double * len(taus))(*[float(t) for t in taus])
        _check(self._lib, self._lib.eife_step_variable(self._g, ctypes.c_void_p(u.data_ptr()), arr, len(taus),
                                                       int(f_kind), float(t0), _stream_ptr(stream)))
        return u

    def profile(self, on):
        """Start (on=True) or stop per-pass event timing; clears the totals."""
        _check(self._lib, self._lib.eife_profile(self._g, 1 if on else 0))

    def profile_read(self):
        """{pass name: (total ms, launches)} since profile(); blocks."""
        ms = (ctypes.c_double * len(PASS_NAMES))()
        cnt = (ctypes.c_int64 * len(PASS_NAMES))()
        _check(self._lib, self._lib.eife_profile_read(self._g, ms, cnt))
        return {PASS_NAMES[k]: (ms[k], cnt[k]) for k in range(len(PASS_NAMES))}

    def norms(self, u, uref=None, stream=None):
        """(L2, H1, max, Allen-Cahn energy) in double; blocks until computed."""
        self._check_array(u, "u")
        ref = None
        if uref is not None:
            self._check_array(uref, "uref")
            ref = ctypes.c_void_p(uref.data_ptr())
        out = (ctypes.c_double * 4)()
        code = self._lib.eife_norms(self._g, ctypes.c_void_p(u.data_ptr()), ref, out, _stream_ptr(stream))
        _check(self._lib, code)
        return tuple(out)

    def norms_noalloc(self, u, uref=None, out=None, stream=None):
        """eife_norms_noalloc: the four values of norms() left in `out`, a float64 CUDA
        tensor of 4 elements (created when None); enqueued on the stream, no wait."""
        self._check_array(u, "u")
        ref = None
        if uref is not None:
            self._check_array(uref, "uref")
            ref = ctypes.c_void_p(uref.data_ptr())
        if out is None:
            out = torch.empty(4, dtype=torch.float64, device=u.device)
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() < 4 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 CUDA tensor of at least 4 elements")
        code = self._lib.eife_norms_noalloc(self._g, ctypes.c_void_p(u.data_ptr()), ref,
                                            ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
        _check(self._lib, code)
        return out

    def energy(self, u, f_kind, stream=None):
        """Discrete energy (D/2) u^T K_1 u + prod(h) sum F(u_i) of the reaction f_kind, in double."""
        self._check_array(u, "u")
        out = ctypes.c_double()
        code = self._lib.eife_energy(self._g, ctypes.c_void_p(u.data_ptr()), int(f_kind), ctypes.byref(out),
                                     _stream_ptr(stream))
        _check(self._lib, code)
        return out.value


class Batch:
    """Independent 2D instances advanced together (eife_create_batch ... eife_batch_step).

    grids: list of (Nx, Ny, hx, hy, D).  The batched nodal array is one
    contiguous 1-D tensor; `offsets` says where instance i starts.
    """

    def __init__(self, grids, dtype="f32"):
        self._lib = load_library()
        self.B = len(grids)
        self.dtype_code, self.torch_dtype = _DTYPES[dtype]
        N = (ctypes.c_int32 * (2 * self.B))(*[int(v) for g in grids for v in g[:2]])
        h = (ctypes.c_double * (2 * self.B))(*[float(v) for g in grids for v in g[2:4]])
        D = (ctypes.c_double * self.B)(*[float(g[4]) for g in grids])
        handle = ctypes.c_void_p()
        _check(self._lib, self._lib.eife_create_batch(self.B, N, h, D, self.dtype_code, ctypes.byref(handle)))
        self._b = handle
        off = (ctypes.c_int64 * (self.B + 1))()
        _check(self._lib, self._lib.eife_batch_offsets(self._b, off))
        self.offsets = list(off)
        self.shapes = [(int(g[1]) - 1, int(g[0]) - 1) for g in grids]

    def close(self):
        if getattr(self, "_b", None):
            self._lib.eife_destroy_batch(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def size(self):
        return self.offsets[-1]

    def set_phi(self, tau, stages):
        _check(self._lib, self._lib.eife_batch_set_phi(self._b, float(tau), int(stages)))

    def autotune(self, cache_path=None, stream=None):
        path = None if cache_path is None else str(cache_path).encode()
        _check(self._lib, self._lib.eife_batch_autotune(self._b, path, _stream_ptr(stream)))

    def class_info(self):
        out, k = [], 0
        buf = (ctypes.c_int32 * 5)()
        while self._lib.eife_batch_class_info(self._b, k, buf) == OK:
            out.append(tuple(buf))
            k += 1
        return out

    def step(self, u, n_steps, f_kind, t0=0.0, stream=None, graph=True):
        """Advance every instance in place; graph=False enqueues on the null stream (no capture)."""
        if not isinstance(u, torch.Tensor) or not u.is_cuda or u.dtype != self.torch_dtype:
            raise TypeError("u must be a CUDA tensor of the batch dtype")
        if not u.is_contiguous() or u.numel() != self.size():
            raise ValueError(f"u must be contiguous with {self.size()} elements")
        sp = _stream_ptr(stream) if graph else ctypes.c_void_p(0)
        _check(self._lib, self._lib.eife_batch_step(self._b, ctypes.c_void_p(u.data_ptr()), int(n_steps),
                                                    int(f_kind), float(t0), sp))
        return u

    def views(self, u):
        """Per-instance 2D views of a batched nodal array."""
        return [u[self.offsets[i]:self.offsets[i + 1]].view(self.shapes[i]) for i in range(self.B)]


CORR_PARAMS = 37889


def _ccheck(lib, code):
    if code != OK:
        raise EIFEError(code, lib.eife_corr_last_error().decode(errors="replace"))


def _f32_dev(x, shape_tail):
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
        raise TypeError("expected a contiguous float32 CUDA tensor")
    if tuple(x.shape[-2:]) != shape_tail:
        raise ValueError(f"expected trailing shape {shape_tail}, got {tuple(x.shape)}")
    return ctypes.c_void_p(x.data_ptr())


class Corrector:
    """Learned corrector (eife_corr_*): a 6-layer 3x3 convolutional network on
    (u_n, u_c) that predicts delta with u_{n+1} = u_c + delta.  Images are
    float32 CUDA tensors of shape (batch, ny, nx) or (ny, nx)."""

    def __init__(self, nx, ny, max_batch=1):
        self._lib = load_library()
        self.nx, self.ny, self.max_batch = int(nx), int(ny), int(max_batch)
        handle = ctypes.c_void_p()
        _ccheck(self._lib, self._lib.eife_corr_create(self.nx, self.ny, self.max_batch, ctypes.byref(handle)))
        self._c = handle

    def close(self):
        if getattr(self, "_c", None):
            self._lib.eife_corr_destroy(self._c)
            self._c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _batch(self, x):
        return 1 if x.dim() == 2 else int(x.shape[0])

    def set_params(self, p):
        import numpy as np
        a = np.ascontiguousarray(p, dtype=np.float32)
        _ccheck(self._lib, self._lib.eife_corr_set_params(
            self._c, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))

    def get_params(self):
        import numpy as np
        a = np.empty(CORR_PARAMS, dtype=np.float32)
        _ccheck(self._lib, self._lib.eife_corr_get_params(
            self._c, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))
        return a

    def set_scale(self, s_out):
        _ccheck(self._lib, self._lib.eife_corr_set_scale(self._c, float(s_out)))

    def set_guard(self, max_change_rms):
        _ccheck(self._lib, self._lib.eife_corr_set_guard(self._c, float(max_change_rms)))

    def set_fused(self, fused):
        """Inference through the one-kernel network (True, default) or one kernel per layer."""
        _ccheck(self._lib, self._lib.eife_corr_set_fused(self._c, 1 if fused else 0))

    def forward(self, un, uc, delta=None, stream=None):
        if delta is None:
            delta = torch.empty_like(uc)
        sh = (self.ny, self.nx)
        _ccheck(self._lib, self._lib.eife_corr_forward(self._c, _f32_dev(un, sh), _f32_dev(uc, sh),
                                                       _f32_dev(delta, sh), self._batch(un), _stream_ptr(stream)))
        return delta

    def grad(self, un, uc, uf, stream=None):
        import numpy as np
        g = np.empty(CORR_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        sh = (self.ny, self.nx)
        _ccheck(self._lib, self._lib.eife_corr_grad(self._c, _f32_dev(un, sh), _f32_dev(uc, sh), _f32_dev(uf, sh),
                                                    self._batch(un), g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                    ctypes.byref(loss), _stream_ptr(stream)))
        return loss.value, g

    def train_step(self, un, uc, uf, lr, want_loss=False, stream=None):
        loss = ctypes.c_double()
        sh = (self.ny, self.nx)
        _ccheck(self._lib, self._lib.eife_corr_train_step(
            self._c, _f32_dev(un, sh), _f32_dev(uc, sh), _f32_dev(uf, sh), self._batch(un), float(lr),
            ctypes.byref(loss) if want_loss else None, _stream_ptr(stream)))
        return loss.value if want_loss else None

    def infer_step(self, coarse, fine, u, t0, fine_steps, theta, stream=None):
        """One corrected step of u in place; returns (fell_back, r, max|u_c + delta|)."""
        fb = ctypes.c_int()
        out2 = (ctypes.c_double * 2)()
        _ccheck(self._lib, self._lib.eife_corr_infer_step(
            self._c, coarse._g, fine._g, _f32_dev(u, (self.ny, self.nx)), float(t0), int(fine_steps), float(theta),
            ctypes.byref(fb), out2, _stream_ptr(stream)))
        return bool(fb.value), out2[0], out2[1]

    def run(self, coarse, fine, u, t0, tau_coarse, n_steps, fine_steps, theta, stream=None):
        """n_steps corrected steps of u in place (native loop); returns the number of fallbacks."""
        fb = ctypes.c_int64()
        _ccheck(self._lib, self._lib.eife_corr_run(
            self._c, coarse._g, fine._g, _f32_dev(u, (self.ny, self.nx)), float(t0), float(tau_coarse),
            int(n_steps), int(fine_steps), float(theta), ctypes.byref(fb), _stream_ptr(stream)))
        return fb.value
