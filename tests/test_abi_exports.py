"""The C-ABI library loads on the CPU and exports every function include/eife.h declares."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eife.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eife_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2209_11922_amd import binding
    path = binding.library_path()
    if not os.path.exists(path):
        from paper_2209_11922_amd import build
        build.build()
    return path


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["eife_create_grid", "eife_set_phi", "eife_step", "eife_destroy_grid", "eife_norms",
                 "eife_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (eife_[a-z0-9_]+)", out))
    assert set(_declared()) <= exported


def test_version_and_error_string_without_gpu(libpath):
    lib = ctypes.CDLL(libpath)
    lib.eife_last_error.restype = ctypes.c_char_p
    assert lib.eife_version() == 1
    assert isinstance(lib.eife_last_error(), bytes)
    # argument validation happens before any device call
    out = ctypes.c_void_p()
    N = (ctypes.c_int32 * 2)(8, 8)
    h = (ctypes.c_double * 2)(0.1, 0.1)
    assert lib.eife_create_grid(4, N, h, ctypes.c_double(1.0), 0, 1, ctypes.byref(out)) == -1
    assert b"d must be" in lib.eife_last_error()
    assert lib.eife_create_grid(2, N, h, ctypes.c_double(1.0), 7, 1, ctypes.byref(out)) == -1  # unknown bc
    assert b"boundary condition" in lib.eife_last_error()
    assert lib.eife_step(None, None, 1, 1, ctypes.c_double(0.0), None) == -1


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2209_11922_amd import binding
    monkeypatch.setattr(binding, "_LIB", None)
    monkeypatch.setattr(binding, "library_path", lambda: str(tmp_path / "libeife.so"))
    with pytest.raises(RuntimeError):
        binding.load_library()


def test_binding_constants_match_the_header():
    """The Python constants carry the values the header's enumerations give."""
    import re
    hdr = open(os.path.join(ROOT, "include", "eife.h")).read()
    vals = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(EIFE_[A-Z0-9_]+)\s*=\s*(-?\d+)", hdr)}
    from paper_2209_11922_amd import binding as b
    pairs = {"F_ZERO": "EIFE_F_ZERO", "F_ALLEN_CAHN": "EIFE_F_ALLEN_CAHN", "F_MMS_U2": "EIFE_F_MMS_U2",
             "F_EX51": "EIFE_F_EX51", "F_CONST": "EIFE_F_CONST", "F_AFFINE_T": "EIFE_F_AFFINE_T",
             "F_FLORY_HUGGINS": "EIFE_F_FLORY_HUGGINS", "F_TRAVELING_WAVE": "EIFE_F_TRAVELING_WAVE",
             "BC_DIRICHLET": "EIFE_BC_DIRICHLET", "BC_PERIODIC": "EIFE_BC_PERIODIC",
             "LOAD_LUMPED": "EIFE_LOAD_LUMPED", "LOAD_NODAL": "EIFE_LOAD_NODAL"}
    for py, c in pairs.items():
        assert getattr(b, py) == vals[c], (py, c)
