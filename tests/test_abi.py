"""The C-ABI library loads and exports every symbol its header declares; host-side
validation answers without touching a GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names.update(re.findall(r"\b(gspca_\w+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_0811_1081_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        from paper_0811_1081_amd import build
        build.build()
    return _binding.load()


def test_header_declares_the_documented_entry_points():
    names = declared_functions()
    for n in ("gspca_fit", "gspca_fit_f32", "gspca_fit_ex", "gspca_workspace_bytes",
              "gspca_status_string", "gspca_default_options", "gspca_version"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_binding_export_list_matches_header():
    from paper_0811_1081_amd import _binding
    assert sorted(_binding.EXPORTS) == declared_functions()


def test_status_strings(lib):
    from paper_0811_1081_amd import _binding as b
    for st in (b.OK, b.NOT_CONVERGED, b.EINVAL, b.EWORKSPACE, b.EDEVICE, b.ENONFINITE, b.ENOMEM):
        assert lib.gspca_status_string(st).decode() != "unknown status"
    assert lib.gspca_status_string(12345).decode() == "unknown status"
    assert lib.gspca_version() >= 100


def _prob(b, M=100, N=20, K=4, dtype=1, X=0x1000, ldx=None):
    return b.Problem(dtype, X, ldx if ldx is not None else M, M, N, K)


def test_workspace_bytes_and_validation_on_host(lib):
    from paper_0811_1081_amd import _binding as b
    op = b.Options()
    lib.gspca_default_options(ctypes.byref(op))
    assert op.algo == b.GS and op.init == b.INIT_MAXNORM and op.max_iter == 10000
    assert abs(op.tol - 1e-7) < 1e-20
    ok = lib.gspca_workspace_bytes(_prob(b), op)
    assert ok > 100 * 20 * 4
    assert lib.gspca_workspace_bytes(_prob(b, dtype=0), op) > ok  # FP64 residual is larger
    for bad in (_prob(b, K=0), _prob(b, K=21), _prob(b, M=0), _prob(b, ldx=50),
                _prob(b, dtype=7), _prob(b, X=0)):
        assert lib.gspca_workspace_bytes(bad, op) == 0
    op2 = b.Options()
    lib.gspca_default_options(ctypes.byref(op2))
    op2.tol = -1.0
    assert lib.gspca_workspace_bytes(_prob(b), op2) == 0
    op2.tol = 1e-6
    op2.max_iter = 0
    assert lib.gspca_workspace_bytes(_prob(b), op2) == 0
    op2.max_iter = 10
    op2.init = b.INIT_GIVEN  # needs T0
    assert lib.gspca_workspace_bytes(_prob(b), op2) == 0


def test_fit_ex_rejects_invalid_arguments_before_any_device_call(lib):
    from paper_0811_1081_amd import _binding as b
    op = b.Options()
    lib.gspca_default_options(ctypes.byref(op))
    res = b.Result(0x1000, 0x2000, 0x3000, None, None, None)
    assert lib.gspca_fit_ex(_prob(b, K=0), op, res, 0x4000, 1 << 30, None) == b.EINVAL
    assert lib.gspca_fit_ex(None, op, res, 0x4000, 1 << 30, None) == b.EINVAL
    empty = b.Result(0, 0, 0, None, None, None)
    assert lib.gspca_fit_ex(_prob(b), op, empty, 0x4000, 1 << 30, None) == b.EINVAL
    # workspace too small is reported before anything is enqueued
    assert lib.gspca_fit_ex(_prob(b), op, res, 0x4000, 16, None) == b.EWORKSPACE
    assert lib.gspca_fit(None, 10, 5, 2, 1e-7, 100, None, None, None, None) == b.EINVAL
    assert lib.gspca_fit_f32(0x1000, 10, 5, 6, 1e-7, 100, 0x1, 0x1, 0x1, None) == b.EINVAL
